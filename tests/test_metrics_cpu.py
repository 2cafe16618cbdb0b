"""Closed-form AQFT accuracy and cutoff selection (host functions of the
library) against the oracle's formula, brute force on small matrices, and
the closed form at the smallest truncation."""

import math

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import qft as Q


@pytest.mark.parametrize("n", [10, 16, 20, 28])
def test_expected_error_matches_oracle_formula(n):
    for k in range(max(0, n - 21), n - 1):
        ref = O.aqft_expected_relerr_gaussian(n, k)
        if ref < 1e-6:
            continue
        # the oracle forms 1 - trace directly, which keeps about 1e-16 / err^2
        # of relative accuracy; the library's form keeps full accuracy
        got = Q.expected_error(n, k)
        assert got == pytest.approx(ref, rel=1e-9 + 4e-16 / ref ** 2), (n, k)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_expected_error_is_frobenius_distance(n):
    # E||(U - U_k) x||^2 / E||U x||^2 = ||U - U_k||_F^2 / N for i.i.d. inputs
    N = 1 << n
    U = O.dft_matrix(N) / math.sqrt(N)
    for k in range(0, n):
        Uk = O.aqft_matrix(n, k)
        brute = float(np.linalg.norm(U - Uk)) / math.sqrt(N)
        assert Q.expected_error(n, k) == pytest.approx(brute, rel=1e-10, abs=1e-15), (n, k)


@pytest.mark.parametrize("n", [4, 10, 20, 28, 31])
def test_smallest_truncation_closed_form(n):
    # k = n - 2 drops the one gate R_n at distance n - 1: error sin(pi / 2^n)
    assert Q.expected_error(n, n - 2) == pytest.approx(math.sin(math.pi / 2 ** n), rel=1e-9)
    assert Q.expected_error(n, n - 1) == 0.0
    assert Q.expected_error(n, -1) == 0.0


def test_expected_error_falls_with_cutoff():
    e = [Q.expected_error(24, k) for k in range(4, 23)]
    assert all(b < a for a, b in zip(e, e[1:]))
    assert Q.expected_error(28, 6) < 0  # M = 21: not evaluated


@pytest.mark.parametrize("n,budget", [(28, 1e-2), (28, 1e-3), (28, 1e-6), (20, 0.05),
                                      (12, 1e-9), (16, 0.0)])
def test_select_cutoff(n, budget):
    k = Q.select_cutoff(n, budget)
    assert Q.expected_error(n, k) <= budget
    if k > max(0, n - 21):
        assert Q.expected_error(n, k - 1) > budget  # the next one down fails
    if budget == 0.0:
        assert k == n - 1


def test_select_cutoff_invalid():
    with pytest.raises(ValueError):
        Q.select_cutoff(28, -1.0)
    with pytest.raises(ValueError):
        Q.select_cutoff(0, 1e-3)
