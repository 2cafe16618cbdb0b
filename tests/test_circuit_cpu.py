"""Grouping of general gate lists into fused passes (host only)."""

import numpy as np
import pytest

from paper_2606_18981_amd import qft as Q

H = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)


def qubits_of(g):
    return {g[1]} if g[0] == "U" else {g[1], g[2]}


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


def random_gates(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = rng.integers(0, 3)
        if kind == 0:
            out.append(("U", int(rng.integers(0, n)), H))
        else:
            a, b = rng.choice(n, 2, replace=False)
            out.append(("CU", int(a), int(b), H) if kind == 1 else ("SWAP", int(a), int(b)))
    return out


@pytest.mark.parametrize("n,B,seed", [(20, 10, 1), (20, 4, 2), (12, 2, 3), (30, 8, 4), (5, 10, 5)])
def test_greedy_grouping(n, B, seed):
    gates = random_gates(n, 200, seed)
    c = build(n, gates)
    begin, tbits = c.describe(B)
    Beff = max(2, min(B, min(n, 12)))
    assert begin[0] == 0 and begin == sorted(begin)
    ends = begin[1:] + [len(gates)]
    for p, (s, e) in enumerate(zip(begin, ends)):
        S = set().union(*(qubits_of(g) for g in gates[s:e]))
        assert len(S) <= Beff
        if e < len(gates):  # greedy: the next gate would not fit
            assert len(S | qubits_of(gates[e])) > Beff
        assert tbits[p] == min(n, 12)
    assert c.info()["passes"] == -1  # describe leaves it uncompiled
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
