"""Plain FP64 oracle for the QFT->FFT transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this file;
only tests, the smoke check and the benchmark's CPU-baseline leg do.  It shares
no code with the HIP path.

Everything here is numpy complex128 / float64 and written to be read against
the paper ("Not Your Usual FFT: QFT->FFT via Classical Quantum-Circuit
Simulation"):

* ``dft_naive`` - the DFT definition, Sec. 2 "From Naive DFT to FFT"
  (DFT_N = [w_N^{k l}], w_N = exp(-2 pi i / N)).
* ``qft_gate_list`` / ``qft_circuit`` - the n-qubit QFT circuit of Fig. 1
  (H on the most significant qubit first, then controlled-R_{d+1} from each
  lower qubit at distance d, final swaps), the AQFT cutoff of Sec. 2
  "Approximate QFT" (keep controlled phases whose control-target distance is
  <= k), and the four methodology steps of Sec. 3 (encode with scale_in,
  build the circuit, evolve, decode to FFT units).
* ``aqft_matrix`` / ``aqft_bins`` - a closed form of the range-k AQFT matrix
  derived from the same circuit (see the function docstring).
* ``qft_fused_targets`` - the same circuit with the commuting controlled
  phases of each target collapsed into one diagonal, the fusion rule of
  Sec. 2 (gate fusion paragraph).  It is the vectorised form used for large n
  and is checked against the gate-by-gate form.
* metrics: relative L2, max error, fidelity and top-bin leakage (Sec. 4).
* ``inverse=True`` everywhere: the same circuit with every controlled phase
  conjugated, R_m -> R_m^* (the e^{+} transform).  The H and swap gates are
  real, so the circuit's matrix becomes its complex conjugate; the QFT and
  AQFT matrices are symmetric, so that is also their adjoint (inverse).

Conventions (readings of the paper):
  - qubit q_j is bit j of the array index (Sec. 2: a 1-wire gate on q_j is
    I_{2^{n-1-j}} (x) U (x) I_{2^j}; Fig. 1: MSB q_{n-1}, LSB q_0);
  - forward sign exp(-2 pi i jk/N) (Sec. 2 definitions of w_N and R_k);
  - norm "unitary" = DFT_N x / sqrt(N) (Sec. 3 step 3), "none" = DFT_N x,
    "inv_n" = DFT_N x / N (Sec. 3 step 4);
  - order "natural" applies the final swaps (output bin k at index k),
    "bitrev" leaves them to the caller (Sec. 3 step 2): out[rev_n(k)] = bin k;
  - cutoff None, < 0 or >= n-1 means the exact QFT; 0 keeps no controlled
    phase (Walsh-Hadamard followed by bit reversal).
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = [
    "NORMS",
    "ORDERS",
    "effective_cutoff",
    "norm_factor",
    "bitrev_index",
    "bitrev_perm",
    "dft_naive",
    "dft_matrix",
    "qft_gate_list",
    "gate_counts",
    "qft_circuit",
    "qft_circuit_matrix",
    "aqft_matrix",
    "aqft_bins",
    "dft_bins",
    "dft_library",
    "qft_fused_targets",
    "qft_state_c",
    "qft_padded",
    "apply_gates",
    "qft_as_gates",
    "rel_l2",
    "max_err",
    "error_norms",
    "fidelity",
    "top_bin_leakage",
    "aqft_error_bound",
    "aqft_expected_relerr_gaussian",
    "c_oracle_available",
    "c_oracle_threads",
]

NORMS = ("unitary", "none", "inv_n")
ORDERS = ("natural", "bitrev")


# ---------------------------------------------------------------------------
# conventions
# ---------------------------------------------------------------------------

def effective_cutoff(n: int, cutoff) -> int:
    """Largest control-target distance kept (Sec. 2, "Approximate QFT").

    k = n-1 is the exact circuit; None, negative values and values >= n-1 are
    read as exact.  k = 0 keeps no controlled phase.
    """
    if n <= 1:
        return 0
    if cutoff is None or cutoff < 0 or cutoff >= n - 1:
        return n - 1
    return int(cutoff)


def norm_factor(n: int, norm: str) -> float:
    """Output scale relative to the unitary QFT (Sec. 3, step 4)."""
    N = 1 << n
    if norm == "unitary":
        return 1.0
    if norm == "none":
        return math.sqrt(N)
    if norm == "inv_n":
        return 1.0 / math.sqrt(N)
    raise ValueError(f"unknown norm {norm!r}")


def bitrev_index(k: int, n: int) -> int:
    """Reverse the n low bits of k (the permutation done by the final swaps)."""
    r = 0
    for _ in range(n):
        r = (r << 1) | (k & 1)
        k >>= 1
    return r


def bitrev_perm(n: int) -> np.ndarray:
    """Array p with p[k] = rev_n(k), built bit by bit."""
    idx = np.arange(1 << n, dtype=np.int64)
    rev = np.zeros_like(idx)
    for b in range(n):
        rev |= ((idx >> b) & 1) << (n - 1 - b)
    return rev


# ---------------------------------------------------------------------------
# the plain definition: naive DFT
# ---------------------------------------------------------------------------

def _omega_table(N: int, inverse: bool = False) -> np.ndarray:
    """w_N^m for m = 0..N-1 with w_N = exp(-2 pi i / N) (Sec. 2); its
    conjugate exp(+2 pi i m / N) for the inverse transform."""
    m = np.arange(N, dtype=np.float64)
    ang = 2.0 * np.pi * m / N
    if inverse:
        return np.cos(ang) + 1j * np.sin(ang)
    return np.cos(ang) - 1j * np.sin(ang)


def dft_matrix(N: int) -> np.ndarray:
    """Unnormalised DFT_N = [w_N^{k l}] (Sec. 2, "From Naive DFT to FFT")."""
    k = np.arange(N, dtype=np.int64)
    return _omega_table(N)[np.outer(k, k) % N]


def dft_naive(x, norm: str = "unitary", order: str = "natural",
              inverse: bool = False) -> np.ndarray:
    """O(N^2) DFT: y_k = s * sum_j x_j w_N^{jk} (Sec. 2 definition).

    The exponent j*k is reduced modulo N in integers before the table lookup,
    so every factor is an FP64 cos/sin of an angle in [0, 2 pi).  s follows
    Sec. 3 step 4: 1/sqrt(N) (unitary), 1 (none), 1/N (inv_n).  inverse=True
    uses w_N^{-jk} (the e^{+} sign).
    """
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = N.bit_length() - 1
    if N != 1 << n:
        raise ValueError("N must be a power of two")
    W = _omega_table(N, inverse)
    j = np.arange(N, dtype=np.int64)
    y = np.empty(N, dtype=np.complex128)
    block = max(1, (1 << 22) // N)
    for k0 in range(0, N, block):
        k = np.arange(k0, min(N, k0 + block), dtype=np.int64)
        y[k0:k0 + k.size] = (W[np.outer(k, j) % N] * x[None, :]).sum(axis=1)
    y *= norm_factor(n, norm) / math.sqrt(N)
    if order == "bitrev":
        out = np.empty_like(y)
        out[bitrev_perm(n)] = y
        return out
    if order != "natural":
        raise ValueError(f"unknown order {order!r}")
    return y


# ---------------------------------------------------------------------------
# the circuit, gate by gate
# ---------------------------------------------------------------------------

def qft_gate_list(n: int, cutoff=None):
    """Gate sequence of the (approximate) QFT circuit.

    Fig. 1 order: for target t from the most significant qubit down, first H
    on t, then controlled-R_{d+1} with control c = t-d for d = 1, 2, ...
    (R_m = diag(1, exp(-2 pi i / 2^m)), Sec. 2 circuit operators).  The range-k
    AQFT keeps only distances d <= k (Sec. 2 "Approximate QFT").  The final
    swaps exchange q_a and q_{n-1-a}.

    Returns a list of tuples ("H", t), ("CR", c, t, m), ("SWAP", a, b).
    """
    k = effective_cutoff(n, cutoff)
    gates = []
    for t in range(n - 1, -1, -1):
        gates.append(("H", t))
        for d in range(1, t + 1):
            if d <= k:
                gates.append(("CR", t - d, t, d + 1))
    for a in range(n // 2):
        gates.append(("SWAP", a, n - 1 - a))
    return gates


def gate_counts(n: int, cutoff=None) -> dict:
    """Numbers of H, controlled-phase and swap gates before any fusion."""
    g = qft_gate_list(n, cutoff)
    return {
        "H": sum(1 for x in g if x[0] == "H"),
        "CR": sum(1 for x in g if x[0] == "CR"),
        "SWAP": sum(1 for x in g if x[0] == "SWAP"),
    }


def _apply_h(psi: np.ndarray, n: int, t: int) -> None:
    """Unit-norm H on qubit t: pairs (i, i + 2^t) with bit t of i clear."""
    v = psi.reshape(1 << (n - 1 - t), 2, 1 << t)
    a = v[:, 0, :].copy()
    b = v[:, 1, :].copy()
    s = 1.0 / math.sqrt(2.0)
    v[:, 0, :] = (a + b) * s
    v[:, 1, :] = (a - b) * s


def _apply_cr(psi: np.ndarray, n: int, c: int, t: int, m: int, conj: bool = False) -> None:
    """Controlled-R_m (or R_m^* when conj): multiply amplitudes whose bits c
    and t are both 1 by exp(-/+ 2 pi i / 2^m)."""
    assert c < t
    v = psi.reshape(1 << (n - 1 - t), 2, 1 << (t - 1 - c), 2, 1 << c)
    v[:, 1, :, 1, :] *= np.exp((2j if conj else -2j) * np.pi / float(1 << m))


def _apply_swap(psi: np.ndarray, n: int, a: int, b: int) -> np.ndarray:
    """Exchange qubits a and b (bit j of the index is numpy axis n-1-j)."""
    v = psi.reshape((2,) * n)
    v = np.swapaxes(v, n - 1 - a, n - 1 - b)
    return np.ascontiguousarray(v).reshape(1 << n)


def qft_circuit(x, cutoff=None, norm: str = "unitary", order: str = "natural",
                encode: bool = True, inverse: bool = False) -> np.ndarray:
    """Gate-by-gate FP64 simulation of the QFT->FFT method (Sec. 3).

    Step 1 (encode): scale_in = ||x||_2, psi = x / scale_in, index i <-> basis
      state |b_{n-1} ... b_0> with q_j = bit j.  A zero input gives zero.
    Step 2 (circuit): ``qft_gate_list`` (swaps only when order == "natural";
      "bitrev" leaves the index permutation to the caller).
    Step 3 (evolve): apply the gates in order.
    Step 4 (decode): multiply by scale_in and by the norm factor.
    inverse=True conjugates every controlled phase (the e^{+} transform).
    """
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = N.bit_length() - 1
    if N != 1 << n:
        raise ValueError("N must be a power of two")
    if order not in ORDERS:
        raise ValueError(f"unknown order {order!r}")
    scale_in = float(np.sqrt(np.sum(np.abs(x) ** 2))) if encode else 1.0
    if scale_in == 0.0:
        return np.zeros(N, dtype=np.complex128)
    psi = x / scale_in
    for g in qft_gate_list(n, cutoff):
        if g[0] == "H":
            _apply_h(psi, n, g[1])
        elif g[0] == "CR":
            _apply_cr(psi, n, g[1], g[2], g[3], inverse)
        elif order == "natural":
            psi = _apply_swap(psi, n, g[1], g[2])
    return psi * (scale_in * norm_factor(n, norm))


def qft_circuit_matrix(n: int, cutoff=None, order: str = "natural",
                       inverse: bool = False) -> np.ndarray:
    """Unitary of the circuit, column by column (small n only)."""
    N = 1 << n
    U = np.empty((N, N), dtype=np.complex128)
    for j in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[j] = 1.0
        U[:, j] = qft_circuit(e, cutoff, "unitary", order, encode=False, inverse=inverse)
    return U


# ---------------------------------------------------------------------------
# closed form of the range-k AQFT
# ---------------------------------------------------------------------------

def aqft_matrix(n: int, cutoff=None, inverse: bool = False) -> np.ndarray:
    """Closed-form range-k AQFT matrix (output in natural order).

    Derivation from Fig. 1: the H on qubit t pairs input bit x_t with output
    bit y_{n-1-t} (the final swaps reverse the qubits) with phase 1/2 of a
    turn, and controlled-R_{d+1} from control c = t-d adds x_c * y_{n-1-t} /
    2^{d+1} turns.  Writing a = c and b = n-1-t, every term is
    x_a y_b 2^{a+b-n} turns with distance d = n-1-a-b, so
        A_k[y, x] = N^{-1/2} exp(-2 pi i sum_{n-1-k <= a+b <= n-1}
                                           x_a y_b 2^{a+b-n}).
    For k = n-1 this is the DFT (terms with a+b >= n are whole turns).
    The condition on a+b is symmetric in (a, b), so A_k is symmetric.
    inverse=True gives the conjugate-phase circuit, conj(A_k).
    """
    k = effective_cutoff(n, cutoff)
    N = 1 << n
    idx = np.arange(N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1  # [index, bit]
    P = np.zeros((N, N), dtype=np.int64)  # phase numerator over 2^n
    for a in range(n):
        for b in range(n):
            if n - 1 - k <= a + b <= n - 1:
                P += np.outer(bits[:, b], bits[:, a]) << (a + b)
    P &= N - 1
    return _omega_table(N, inverse)[P] / math.sqrt(N)


def _aqft_bin_coeffs(n: int, k: int, y: int) -> list:
    """C_a(y) with phase(x, y) = sum_a x_a C_a(y) / 2^n turns (mod 1)."""
    N = 1 << n
    C = []
    for a in range(n):
        c = 0
        for b in range(n):
            if n - 1 - k <= a + b <= n - 1 and (y >> b) & 1:
                c += 1 << (a + b)
        C.append(c & (N - 1))
    return C


def aqft_bins(x, bins, cutoff=None, norm: str = "unitary", inverse: bool = False) -> np.ndarray:
    """Selected outputs (natural order) of the closed-form AQFT, O(N) per bin.

    Uses the C helper when it is built (large N), else numpy.  The inverse
    (conjugate-phase) outputs are conj(A_k conj(x)), an exact identity since
    the norm factors are real.
    """
    if inverse:
        return np.conj(aqft_bins(np.conj(np.asarray(x, dtype=np.complex128)), bins, cutoff, norm))
    x = np.ascontiguousarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = N.bit_length() - 1
    k = effective_cutoff(n, cutoff)
    bins = np.asarray(bins, dtype=np.int64)
    lib = _c_lib()
    scale = norm_factor(n, norm) / math.sqrt(N)
    if lib is not None and N >= (1 << 12):
        out = np.empty(bins.size, dtype=np.complex128)
        lib.oracle_aqft_bins(
            x.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(n), ctypes.c_int(k),
            bins.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(bins.size),
            out.ctypes.data_as(ctypes.c_void_p))
        return out * scale
    W = _omega_table(N)
    out = np.empty(bins.size, dtype=np.complex128)
    for i, y in enumerate(bins.tolist()):
        C = _aqft_bin_coeffs(n, k, y)
        ph = np.zeros(1, dtype=np.int64)
        for a in range(n):  # phase for all x, built one input bit at a time
            ph = np.concatenate([ph, (ph + C[a]) & (N - 1)])
        out[i] = np.sum(x * W[ph])
    return out * scale


def dft_bins(x, bins, norm: str = "unitary", inverse: bool = False) -> np.ndarray:
    """Selected outputs y_k = s sum_j x_j w_N^{jk mod N} of the exact DFT
    (w_N^{-jk} when inverse, computed as conj of the forward sums of conj x)."""
    if inverse:
        return np.conj(dft_bins(np.conj(np.asarray(x, dtype=np.complex128)), bins, norm))
    x = np.ascontiguousarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = N.bit_length() - 1
    bins = np.asarray(bins, dtype=np.int64)
    lib = _c_lib()
    scale = norm_factor(n, norm) / math.sqrt(N)
    if lib is not None and N >= (1 << 12):
        out = np.empty(bins.size, dtype=np.complex128)
        lib.oracle_dft_bins(
            x.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(n),
            bins.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(bins.size),
            out.ctypes.data_as(ctypes.c_void_p))
        return out * scale
    W = _omega_table(N)
    j = np.arange(N, dtype=np.int64)
    out = np.array([np.sum(x * W[(j * kk) % N]) for kk in bins.tolist()],
                   dtype=np.complex128)
    return out * scale


def dft_library(x, norm: str = "unitary", order: str = "natural", workers: int = -1,
                inverse: bool = False):
    """The exact DFT through a library FFT (scipy.fft, FP64), for full-size
    references at large N.  The library routine is the special case that
    tests/test_oracle.py checks against ``dft_naive``.  inverse=True uses the
    library inverse FFT times N (the unnormalised e^{+} sums)."""
    import scipy.fft
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = N.bit_length() - 1
    y = scipy.fft.ifft(x, workers=workers) * N if inverse else scipy.fft.fft(x, workers=workers)
    y *= norm_factor(n, norm) / math.sqrt(N)
    if order == "bitrev":
        out = np.empty_like(y)
        out[bitrev_perm(n)] = y
        return out
    return y


# ---------------------------------------------------------------------------
# per-target fused form (vectorised, for large n)
# ---------------------------------------------------------------------------

def qft_fused_targets(x, cutoff=None, norm: str = "unitary",
                      order: str = "natural", inverse: bool = False) -> np.ndarray:
    """The circuit with the controlled phases of each target fused.

    Sec. 2 (gate fusion): commuting diagonal factors collapse into one
    diagonal.  For target t the kept controlled-R_{d+1} (controls c = t-d,
    d <= k) all act on amplitudes with bit t = 1 and multiply them by
    exp(-2 pi i sum_c b_c 2^c / 2^{t+1}), i.e. by w_{2^{t+1}}^u where u is
    (i mod 2^t) with the bits below t-k cleared.  With the final swaps this is
    the radix-2 decimation-in-frequency FFT of Sec. 2 ("From FFT to QFT") with
    unit-norm butterflies and a truncated twiddle index.

    No scale_in normalisation is applied here (the map is linear).
    inverse=True conjugates every twiddle (the conjugate-phase circuit).
    """
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = N.bit_length() - 1
    k = effective_cutoff(n, cutoff)
    psi = x.copy()
    s = 1.0 / math.sqrt(2.0)
    for t in range(n - 1, -1, -1):
        v = psi.reshape(1 << (n - 1 - t), 2, 1 << t)
        a = v[:, 0, :].copy()
        b = v[:, 1, :].copy()
        u = np.arange(1 << t, dtype=np.int64)
        low = max(0, t - k)
        u = (u >> low) << low
        tw = np.exp((2j if inverse else -2j) * np.pi * u.astype(np.float64) / float(1 << (t + 1)))
        v[:, 0, :] = (a + b) * s
        v[:, 1, :] = (a - b) * s * tw[None, :]
    psi *= norm_factor(n, norm)
    if order == "natural":
        return psi[bitrev_perm(n)]
    if order != "bitrev":
        raise ValueError(f"unknown order {order!r}")
    return psi


def qft_state_c(x, cutoff=None, norm: str = "unitary", order: str = "natural",
                inverse: bool = False) -> np.ndarray:
    """``qft_fused_targets`` computed by the plain C helper (qft_state.c):
    the same per-target steps (H on qubit t, then the collapsed controlled
    phases of target t), with the pairs of each target split over OpenMP
    threads, for whole outputs at n = 28-31 in seconds.  Needs the built C
    helper (oracle/build_oracle.py); raises if it is missing."""
    lib = _c_lib()
    if lib is None:
        raise RuntimeError("the oracle's C helper is not built (python -m oracle.build_oracle)")
    if order not in ORDERS:
        raise ValueError(f"unknown order {order!r}")
    psi = np.array(x, dtype=np.complex128, copy=True, order="C")
    N = psi.shape[0]
    n = N.bit_length() - 1
    if N != 1 << n:
        raise ValueError("N must be a power of two")
    k = effective_cutoff(n, cutoff)
    out = np.empty_like(psi) if order == "natural" else None
    lib.oracle_qft_state(
        psi.ctypes.data_as(ctypes.c_void_p),
        out.ctypes.data_as(ctypes.c_void_p) if out is not None else None,
        ctypes.c_int(n), ctypes.c_int(k), ctypes.c_int(1 if inverse else 0),
        ctypes.c_double(norm_factor(n, norm)))
    if out is None:
        return psi
    del psi
    return out


def qft_padded(x, cutoff=None, norm: str = "unitary", order: str = "natural",
               inverse: bool = False) -> np.ndarray:
    """Sec. 3 step 1 for a length N that is not a power of two: n = ceil(log2 N)
    qubits, 2^n amplitudes, the input followed by zeros; the result is the
    (approximate) DFT of length 2^n of that padded input."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = max(0, (N - 1).bit_length())
    padded = np.zeros(1 << n, dtype=np.complex128)
    padded[:N] = x
    return qft_circuit(padded, cutoff, norm, order, encode=True, inverse=inverse)


def apply_gates(x, gates) -> np.ndarray:
    """Gate-by-gate FP64 simulation of a general gate list on n qubits, with
    the Sec. 2 conventions (qubit q_j = bit j of the index; a one-wire gate U
    on q_j is I_{2^{n-1-j}} (x) U (x) I_{2^j}).  Gates:
      ("U", q, M)      2x2 matrix M on qubit q;
      ("CU", c, t, M)  M on qubit t where qubit c is 1;
      ("SWAP", a, b)   exchange qubits a and b.
    """
    psi = np.array(x, dtype=np.complex128)
    N = psi.shape[0]
    n = N.bit_length() - 1
    for g in gates:
        if g[0] == "U":
            q, M = g[1], np.asarray(g[2], dtype=np.complex128)
            v = psi.reshape(1 << (n - 1 - q), 2, 1 << q)
            a = v[:, 0, :].copy()
            b = v[:, 1, :].copy()
            v[:, 0, :] = M[0, 0] * a + M[0, 1] * b
            v[:, 1, :] = M[1, 0] * a + M[1, 1] * b
        elif g[0] == "CU":
            c, t, M = g[1], g[2], np.asarray(g[3], dtype=np.complex128)
            v = psi.reshape((2,) * n)  # axis n-1-j holds bit j
            sel = [slice(None)] * n
            sel[n - 1 - c] = 1
            sub = v[tuple(sel)]  # control bit fixed to 1: n-1 axes
            ax = (n - 1 - t) - (1 if (n - 1 - c) < (n - 1 - t) else 0)
            s0 = [slice(None)] * (n - 1)
            s1 = [slice(None)] * (n - 1)
            s0[ax] = 0
            s1[ax] = 1
            a = sub[tuple(s0)].copy()
            b = sub[tuple(s1)].copy()
            sub[tuple(s0)] = M[0, 0] * a + M[0, 1] * b
            sub[tuple(s1)] = M[1, 0] * a + M[1, 1] * b
        elif g[0] == "SWAP":
            psi = _apply_swap(psi, n, g[1], g[2])
        else:
            raise ValueError(f"unknown gate {g[0]!r}")
    return psi


def qft_as_gates(n: int, cutoff=None, order: str = "natural"):
    """The QFT circuit of ``qft_gate_list`` written as general gates: H as the
    matrix [[1, 1], [1, -1]] / sqrt(2), controlled-R_m as controlled
    diag(1, exp(-2 pi i / 2^m)), and the swaps (natural order only)."""
    h = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)
    out = []
    for g in qft_gate_list(n, cutoff):
        if g[0] == "H":
            out.append(("U", g[1], h))
        elif g[0] == "CR":
            out.append(("CU", g[1], g[2], np.diag([1.0, np.exp(-2j * np.pi / float(1 << g[3]))])))
        elif order == "natural":
            out.append(("SWAP", g[1], g[2]))
    return out


# ---------------------------------------------------------------------------
# metrics (Sec. 4) and AQFT error formulas
# ---------------------------------------------------------------------------

def rel_l2(y, ref) -> float:
    """||y - ref||_2 / ||ref||_2 (0 if both are zero)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    d = float(np.linalg.norm(y - ref))
    r = float(np.linalg.norm(ref))
    return d / r if r > 0 else d


def max_err(y, ref) -> float:
    """max_k |y_k - ref_k| over the RMS amplitude of ref."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    rms = float(np.linalg.norm(ref)) / math.sqrt(max(1, ref.size))
    m = float(np.max(np.abs(y - ref))) if y.size else 0.0
    return m / rms if rms > 0 else m


def error_norms(y, ref, chunk: int = 1 << 24) -> dict:
    """``rel_l2`` and ``max_err`` of y against ref in one pass over chunks of
    both arrays (for 2^28-2^31-element outputs, without full-size FP64
    temporaries).  Sums of squares are accumulated in FP64."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    if y.shape != ref.shape:
        raise ValueError("shape mismatch")
    d2 = 0.0
    r2 = 0.0
    m = 0.0
    for i in range(0, ref.size, chunk):
        a = y[i:i + chunk].astype(np.complex128)
        b = ref[i:i + chunk].astype(np.complex128)
        e = np.abs(a - b)
        d2 += float(np.dot(e, e))
        r2 += float(np.vdot(b, b).real)
        if e.size:
            m = max(m, float(np.max(e)))
    rn = math.sqrt(r2)
    rms = rn / math.sqrt(max(1, ref.size))
    return {"rel_l2": math.sqrt(d2) / rn if rn > 0 else math.sqrt(d2),
            "max_err": m / rms if rms > 0 else m}


def fidelity(y, ref) -> float:
    """Squared normalised inner product |<ref, y>|^2 / (|ref|^2 |y|^2) (Sec. 4)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = abs(np.vdot(ref, y)) ** 2
    den = float(np.vdot(ref, ref).real) * float(np.vdot(y, y).real)
    return float(num / den)


def top_bin_leakage(y, ref) -> float:
    """1 - |y_{k*}|^2 / ||y||^2 with k* = argmax |ref| (lowest on ties) (Sec. 4)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    kstar = int(np.argmax(np.abs(ref)))
    return float(1.0 - abs(y[kstar]) ** 2 / float(np.vdot(y, y).real))


def aqft_error_bound(n: int, cutoff) -> float:
    """Operator-norm bound ||U - U_k||_2 <= sum over dropped gates of ||R - I||.

    Each dropped controlled-R_{d+1} differs from I by |1 - e^{-i theta}| =
    2 sin(theta / 2) with theta = 2 pi / 2^{d+1}; there are n-d gates at
    distance d (Sec. 2, "Approximate QFT").
    """
    k = effective_cutoff(n, cutoff)
    return float(sum((n - d) * 2.0 * math.sin(math.pi / 2.0 ** (d + 1))
                     for d in range(k + 1, n)))


def aqft_expected_relerr_gaussian(n: int, cutoff) -> float:
    """Expected rel-L2 of the AQFT vs the DFT for i.i.d. complex Gaussian x.

    E||(U - U_k)x||^2 / E||U x||^2 = ||U - U_k||_F^2 / N.
    By the closed form (``aqft_matrix``) U_k[y,x] = U[y,x] e^{2 pi i D(x,y)}
    with D the dropped terms sum_{a+b <= n-2-k} x_a y_b 2^{a+b-n}, so
    ||U - U_k||_F^2 / N = 2 (1 - N^{-2} sum_{x,y} cos 2 pi D(x,y)).  Only
    input bits a < M = n-1-k and output bits b < M appear in D; summing over
    the input bits factor by factor gives
        N^{-2} sum_{x,y} e^{2 pi i D} = 2^{-M} sum_{y<2^M} prod_{a<M} (1 + e^{i theta_a(y)}) / 2,
    theta_a(y) = 2 pi (y mod 2^{M-a}) 2^{a-n}.
    """
    k = effective_cutoff(n, cutoff)
    M = n - 1 - k
    if M <= 0:
        return 0.0
    y = np.arange(1 << M, dtype=np.int64)
    prod = np.ones(1 << M, dtype=np.complex128)
    for a in range(M):
        th = 2.0 * np.pi * (y % (1 << (M - a))).astype(np.float64) * 2.0 ** (a - n)
        prod *= (1.0 + np.exp(1j * th)) / 2.0
    tr = float(np.mean(prod).real)
    return math.sqrt(max(0.0, 2.0 * (1.0 - tr)))


# ---------------------------------------------------------------------------
# optional C helper for O(N)-per-bin sums at large N
# ---------------------------------------------------------------------------

_LIB = None
_LIB_TRIED = False


def _c_lib():
    global _LIB, _LIB_TRIED
    if _LIB_TRIED:
        return _LIB
    _LIB_TRIED = True
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboracle_bins.so")
    if os.path.exists(path):
        lib = ctypes.CDLL(path)
        lib.oracle_dft_bins.restype = None
        lib.oracle_aqft_bins.restype = None
        lib.oracle_qft_state.restype = None
        lib.oracle_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def c_oracle_available() -> bool:
    return _c_lib() is not None


def c_oracle_threads() -> int:
    """Threads the C helper's parallel loops use (OpenMP maximum)."""
    lib = _c_lib()
    return int(lib.oracle_threads()) if lib is not None else 0
