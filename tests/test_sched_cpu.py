"""The request server's scheduler on a simulated device (CPU only).

The same admission loop that drives the GPU runs here against a virtual
clock, where request i occupies bytes[i] of the HBM budget for service[i]
seconds once admitted.
"""

import numpy as np
import pytest

from paper_2606_18981_amd import serve as S
from paper_2606_18981_amd import qft as Q


def _check_invariants(res, budget, max_inflight, nbytes):
    ok = res["status"] == 0
    adm, comp = res["admitted"], res["completed"]
    # FIFO admission: admission times follow request order
    assert np.all(np.diff(adm) >= 0)
    assert np.all(adm >= res["arrival"] - 1e-12)
    assert np.all(comp[ok] >= adm[ok])
    # budget and slots respected at every admission instant
    for i in np.nonzero(ok)[0]:
        t = adm[i]
        live = ok & (adm <= t) & (comp > t)
        assert live.sum() <= max_inflight
        assert nbytes[live].sum() <= budget


def test_no_contention_runs_immediately():
    arr = np.linspace(0, 1, 50)
    sv = np.full(50, 0.01)
    nb = np.full(50, 10)
    res, st = S.simulate(1000, 8, arr, nb, sv)
    assert np.allclose(res["admitted"], arr)
    assert np.allclose(res["completed"], arr + sv)
    assert st["completed"] == 50 and st["failed"] == 0
    assert st["peak_inflight"] == 1


def test_single_slot_is_fifo_queue():
    # one in-flight slot: completion_i = max(arrival_i, completion_{i-1}) + s_i
    rng = np.random.default_rng(1)
    arr = np.cumsum(rng.exponential(0.01, 200))
    sv = rng.exponential(0.012, 200)
    nb = np.ones(200, dtype=np.int64)
    res, st = S.simulate(10, 1, arr, nb, sv)
    c = 0.0
    for i in range(200):
        c = max(arr[i], c) + sv[i]
        assert res["completed"][i] == pytest.approx(c)
    _check_invariants(res, 10, 1, nb)


def test_budget_limits_concurrency():
    # 10 requests arriving together, each half the budget: two run at a time
    arr = np.zeros(10)
    sv = np.full(10, 1.0)
    nb = np.full(10, 50)
    res, st = S.simulate(100, 64, arr, nb, sv)
    assert st["peak_inflight"] == 2
    assert st["peak_reserved_bytes"] == 100
    assert np.allclose(res["completed"], np.repeat(np.arange(1, 6), 2))
    _check_invariants(res, 100, 64, nb)


def test_oversized_request_fails_others_proceed():
    arr = np.array([0.0, 0.1, 0.2])
    sv = np.array([0.5, 0.5, 0.5])
    nb = np.array([10, 1000, 10])
    res, st = S.simulate(100, 4, arr, nb, sv)
    assert res["status"][1] == Q.QFT_ERR_BUSY
    assert res["status"][0] == 0 and res["status"][2] == 0
    assert st["failed"] == 1 and st["completed"] == 2
    assert res["admitted"][2] == pytest.approx(0.2)


def test_head_of_line_waits_for_memory():
    # a big request at the head blocks later small ones until memory frees
    arr = np.array([0.0, 0.1, 0.2, 0.3])
    sv = np.array([1.0, 1.0, 0.1, 0.1])
    nb = np.array([60, 60, 10, 10])
    res, st = S.simulate(100, 8, arr, nb, sv)
    assert res["admitted"][1] == pytest.approx(1.0)
    assert res["admitted"][2] == pytest.approx(1.0)
    assert res["admitted"][3] == pytest.approx(1.0)
    _check_invariants(res, 100, 8, nb)


@pytest.mark.parametrize("slots", [1, 2, 4, 16])
def test_random_traces_respect_limits(slots):
    rng = np.random.default_rng(slots)
    m = 500
    arr = np.cumsum(rng.exponential(0.001, m))
    sv = rng.exponential(0.004, m)
    nb = rng.integers(1, 60, m)
    res, st = S.simulate(120, slots, arr, nb, sv)
    assert st["completed"] == m
    _check_invariants(res, 120, slots, nb)
    summ = S.latency_summary(res)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0


def test_more_slots_never_hurt_latency_here():
    rng = np.random.default_rng(7)
    m = 400
    arr = np.cumsum(rng.exponential(0.002, m))
    sv = rng.exponential(0.003, m)
    nb = np.ones(m, dtype=np.int64)
    r1, _ = S.simulate(10 ** 6, 1, arr, nb, sv)
    r8, _ = S.simulate(10 ** 6, 8, arr, nb, sv)
    assert np.percentile(r8["latency"], 99) <= np.percentile(r1["latency"], 99)


def test_invalid_arguments():
    with pytest.raises(Q.QftError):
        S.simulate(100, 0, [0.0], [1], [1.0])
    with pytest.raises(Q.QftError):
        S.simulate(100, 1, [1.0, 0.5], [1, 1], [1.0, 1.0])
