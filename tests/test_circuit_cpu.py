"""Grouping of general gate lists into fused passes (host only)."""

import numpy as np
import pytest

from paper_2606_18981_amd import qft as Q

H = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)


def is_diag(u):
    u = np.asarray(u)
    return u[0, 1] == 0 and u[1, 0] == 0


def qubits_of(g):
    """The qubits a gate needs in its pass's tile: those whose amplitudes it
    mixes (controls and diagonal gates only select or scale)."""
    if g[0] == "SWAP":
        return {g[1], g[2]}
    if g[0] == "U":
        return set() if is_diag(g[2]) else {g[1]}
    return set() if is_diag(g[3]) else {g[2]}


def build(n, gates, dtype="c64"):
    c = Q.Circuit(n, dtype)
    for g in gates:
        if g[0] == "U":
            c.add_1q(g[1], g[2])
        elif g[0] == "CU":
            c.add_controlled(g[1], g[2], g[3])
        else:
            c.add_swap(g[1], g[2])
    return c


PHASE = np.diag([1.0, np.exp(0.7j)])


def random_gates(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = rng.integers(0, 5)
        if kind == 0:
            out.append(("U", int(rng.integers(0, n)), H))
        elif kind == 1:
            out.append(("U", int(rng.integers(0, n)), PHASE))
        else:
            a, b = rng.choice(n, 2, replace=False)
            if kind == 2:
                out.append(("CU", int(a), int(b), H))
            elif kind == 3:
                out.append(("CU", int(a), int(b), PHASE))
            else:
                out.append(("SWAP", int(a), int(b)))
    return out


def tile_size(n, dtype):
    return min(n, 13 if dtype == "c64" else 12)


@pytest.mark.parametrize("n,B,seed,dtype", [(20, 10, 1, "c64"), (20, 4, 2, "c64"),
                                            (12, 2, 3, "c128"), (30, 8, 4, "c64"),
                                            (5, 10, 5, "c128"), (24, 0, 6, "c64"),
                                            (24, 0, 7, "c128")])
def test_greedy_grouping(n, B, seed, dtype):
    gates = random_gates(n, 200, seed)
    c = build(n, gates, dtype)
    begin, tbits = c.describe(B)
    T = tile_size(n, dtype)
    default = T - (3 if dtype == "c64" else 2)
    Beff = max(2, min(B if B > 0 else default, T))
    assert begin[0] == 0 and begin == sorted(begin)
    ends = begin[1:] + [len(gates)]
    for p, (s, e) in enumerate(zip(begin, ends)):
        S = set().union(*(qubits_of(g) for g in gates[s:e]))
        assert len(S) <= Beff
        if e < len(gates):  # greedy: the next gate would not fit
            assert len(S | qubits_of(gates[e])) > Beff
        assert tbits[p] == T
    assert c.info()["passes"] == -1  # describe leaves it uncompiled
    c.close()


def test_diagonal_gates_and_controls_need_no_tile_qubit():
    """Controlled phases, one-qubit phases and the controls of non-diagonal
    gates ride along in any pass: the QFT as general gates needs one pass
    per B Hadamard targets, plus the passes its swaps need."""
    n = 24
    c = Q.Circuit(n, "c64")
    for t in range(n - 1, -1, -1):
        c.add_1q(t, H)
        for d in range(1, t + 1):
            c.add_controlled(t - d, t, np.diag([1.0, np.exp(-2j * np.pi / 2.0 ** (d + 1))]))
    begin, _ = c.describe(12)
    # H targets 23..12 and 11..0 in two passes; the 12 swaps need 24 qubits
    assert len(begin) == 2
    for a in range(n // 2):
        c.add_swap(a, n - 1 - a)
    begin, _ = c.describe(12)
    assert len(begin) == 4
    c.close()
    # a run of diagonal gates alone fits in one pass however many qubits it has
    c = Q.Circuit(30, "c64")
    for q in range(30):
        c.add_1q(q, PHASE)
        c.add_controlled(q, (q + 7) % 30, PHASE)
    c.add_controlled(3, 29, H)  # control 3 need not be in the tile
    assert c.describe(2)[0] == [0]
    c.close()


def test_circuit_errors():
    with pytest.raises(Q.QftError):
        Q.Circuit(0)
    c = Q.Circuit(4)
    with pytest.raises(Q.QftError):
        c.add_1q(4, H)
    with pytest.raises(Q.QftError):
        c.add_controlled(2, 2, H)
    with pytest.raises(Q.QftError):
        c.add_swap(1, 9)
    assert c.describe() == ([], [])
    c.close()
