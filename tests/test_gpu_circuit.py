"""General fused circuits on the GPU against the oracle's gate-by-gate
simulation: random gate lists and the QFT written as general gates."""

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

def within(y, ref, tol):
    """Relative L2 and max error over the RMS amplitude both <= tol."""
    e = O.error_norms(y, ref)
    return e["rel_l2"] <= tol and e["max_err"] <= tol


TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_18981_amd import qft as Q
    return torch, Q


def unitary(rng):
    q, _ = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
    return q


def random_gates(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = rng.integers(0, 3) if n > 1 else 0
        if kind == 0:
            out.append(("U", int(rng.integers(0, n)), unitary(rng)))
        else:
            a, b = rng.choice(n, 2, replace=False)
            out.append(("CU", int(a), int(b), unitary(rng)) if kind == 1
                       else ("SWAP", int(a), int(b)))
    return out


def run(torch, Q, n, gates, x, dtype, B=0):
    c = Q.Circuit(n, dtype)
    for g in gates:
        if g[0] == "U":
            c.add_1q(g[1], g[2])
        elif g[0] == "CU":
            c.add_controlled(g[1], g[2], g[3])
        else:
            c.add_swap(g[1], g[2])
    c.compile(B)
    t = torch.from_numpy(x.astype(NPDT[dtype])).cuda()
    c.execute(t)
    torch.cuda.synchronize()
    info = c.info()
    c.close()
    return t.cpu().numpy().astype(np.complex128), info


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,count,B", [(1, 5, 0), (5, 40, 0), (12, 150, 6), (16, 300, 0),
                                       (20, 200, 10), (13, 100, 2)])
def test_random_circuits(env, dtype, n, count, B):
    torch, Q = env
    print(f"[gpu] circuit n={n} gates={count} B={B} {dtype}", flush=True)
    gates = random_gates(n, count, 9000 + n)
    x = I.gaussian(n, 9100 + n)
    y, info = run(torch, Q, n, gates, x, dtype, B)
    assert info["gates"] == len(gates) and info["passes"] >= 1
    assert within(y, O.apply_gates(x, gates), TOL[dtype])


def diagonal(rng):
    """A diagonal 2x2 with entries of modulus near 1 (not unitary)."""
    return np.diag(rng.uniform(0.9, 1.1, 2) * np.exp(1j * rng.uniform(0, 2 * np.pi, 2)))


def phase(rng):
    """diag(1, e^{i phi}): a phase gate."""
    return np.diag([1.0, np.exp(1j * rng.uniform(-np.pi, np.pi))])


def mixed_gates(n, count, seed):
    """Non-diagonal, diagonal and phase one-qubit gates, controlled gates of
    all three kinds and swaps, on qubits anywhere in the register."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = rng.integers(0, 7) if n > 1 else rng.integers(0, 2)
        if kind == 0:
            out.append(("U", int(rng.integers(0, n)), unitary(rng)))
        elif kind == 1:
            out.append(("U", int(rng.integers(0, n)), diagonal(rng)))
        elif kind == 5:
            out.append(("U", int(rng.integers(0, n)), phase(rng)))
        elif kind == 6:
            a, b = rng.choice(n, 2, replace=False)
            out.append(("CU", int(a), int(b), phase(rng)))
        else:
            a, b = rng.choice(n, 2, replace=False)
            if kind == 2:
                out.append(("CU", int(a), int(b), unitary(rng)))
            elif kind == 3:
                out.append(("CU", int(a), int(b), diagonal(rng)))
            else:
                out.append(("SWAP", int(a), int(b)))
    return out


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,count,B", [(1, 6, 0), (4, 60, 0), (7, 80, 3), (13, 200, 0),
                                       (14, 200, 4), (17, 300, 0), (21, 250, 9)])
def test_mixed_diagonal_circuits(env, dtype, n, count, B):
    """Diagonal runs split over the low and high factor tables and the
    per-element list, controls inside and outside the tile."""
    torch, Q = env
    print(f"[gpu] mixed circuit n={n} gates={count} B={B} {dtype}", flush=True)
    gates = mixed_gates(n, count, 9300 + n)
    x = I.gaussian(n, 9400 + n)
    y, info = run(torch, Q, n, gates, x, dtype, B)
    assert info["gates"] == len(gates)
    assert within(y, O.apply_gates(x, gates), TOL[dtype])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_diagonal_only_circuit_is_one_pass(env, dtype):
    torch, Q = env
    n = 20
    rng = np.random.default_rng(9500)
    gates = []
    for q in range(n):
        gates.append(("U", q, diagonal(rng)))
        gates.append(("CU", q, (q + 1 + int(rng.integers(0, n - 1))) % n, diagonal(rng)))
    gates = [g for g in gates if g[0] == "U" or g[1] != g[2]]
    x = I.gaussian(n, 9501)
    y, info = run(torch, Q, n, gates, x, dtype)
    assert info["passes"] == 1
    assert within(y, O.apply_gates(x, gates), TOL[dtype])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,k", [(10, None), (18, 6)])
def test_qft_as_general_circuit(env, dtype, n, k):
    torch, Q = env
    print(f"[gpu] qft as circuit n={n} k={k} {dtype}", flush=True)
    x = I.gaussian(n, 9200 + n)
    y, info = run(torch, Q, n, O.qft_as_gates(n, k), x, dtype)
    ref = O.qft_fused_targets(x, k)
    assert within(y, ref, TOL[dtype])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_empty_and_swap_only_circuits(env, dtype):
    """No gates: no pass, the state is untouched.  Only swaps: a permutation
    of the amplitudes, exact to the bit."""
    torch, Q = env
    n = 15
    x = I.gaussian(n, 9600)
    y, info = run(torch, Q, n, [], x, dtype)
    assert info["passes"] == 0
    assert np.array_equal(y, x.astype(NPDT[dtype]).astype(np.complex128))
    gates = [("SWAP", a, n - 1 - a) for a in range(n // 2)] + [("SWAP", 0, 7), ("SWAP", 3, 14)]
    y, info = run(torch, Q, n, gates, x, dtype)
    ref = O.apply_gates(x.astype(NPDT[dtype]).astype(np.complex128), gates)
    assert np.array_equal(y, ref)
