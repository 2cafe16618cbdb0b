"""GPU tests of the request server: every result is the same alone and in
the mix (bitwise: same kernels and plans) and matches the oracle on the
host-regenerated Philox input."""

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

def within(y, ref, tol):
    """Relative L2 and max error over the RMS amplitude both <= tol."""
    e = O.error_norms(y, ref)
    return e["rel_l2"] <= tol and e["max_err"] <= tol


TOL = {0: 1e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2606_18981_amd import qft as Q
    from paper_2606_18981_amd import serve as S
    assert torch.cuda.is_available()
    return torch, Q, S


def test_served_results_equal_alone_and_oracle(env):
    torch, Q, S = env
    trace = I.served_trace(1005, rate=2000.0, duration=0.15, n_lo=10, n_hi=18)
    m = len(trace["arrival"])
    # bunch half of the arrivals at t = 0 so that requests overlap
    trace["arrival"][: m // 2] = 0.0
    trace["arrival"] = np.sort(trace["arrival"])
    print(f"[gpu] served trace of {m} requests", flush=True)
    outs = []
    for i in range(m):
        dt = torch.complex128 if trace["dtype"][i] else torch.complex64
        outs.append(torch.empty(1 << int(trace["n"][i]), dtype=dt, device="cuda"))
    reqs = S.requests_from_trace(trace, outs=outs)
    srv = S.Server(budget_bytes=8 << 30, max_inflight=32, num_streams=4)
    res, st = srv.run(reqs)
    torch.cuda.synchronize()
    assert st["completed"] == m and st["failed"] == 0
    assert st["peak_inflight"] > 1
    assert np.all(res["completed"] >= res["admitted"])
    plans = {}
    for i in range(m):
        n, k, dt, seed = (int(trace["n"][i]), int(trace["cutoff"][i]), int(trace["dtype"][i]),
                          int(trace["seed"][i]))
        key = (n, k, dt)
        if key not in plans:
            plans[key] = Q.Plan(n, k, "unitary", "c128" if dt else "c64")
        t = torch.empty_like(outs[i])
        Q.fill_random(t, "gaussian", seed=seed, stream_id=0)
        plans[key].execute(t)
        torch.cuda.synchronize()
        assert torch.equal(t, outs[i]), f"request {i} differs alone vs in the mix"
        if i % 8 == 0:
            x = I.philox_gaussian(n, seed, 0)
            ref = O.qft_fused_targets(x, None if k < 0 else k)
            y = outs[i].cpu().numpy().astype(np.complex128)
            assert within(y, ref, TOL[dt])
    srv.close()
    for p in plans.values():
        p.close()


def test_budget_admission_on_gpu(env):
    torch, Q, S = env
    # 12 requests of n = 20 complex64 (8 MiB state each) with a 20 MiB budget:
    # at most two in flight at once
    trace = {"arrival": np.zeros(12), "n": np.full(12, 20), "dtype": np.zeros(12, int),
             "cutoff": np.full(12, -1), "seed": np.arange(1, 13)}
    reqs = S.requests_from_trace(trace, order="bitrev")
    srv = S.Server(budget_bytes=20 << 20, max_inflight=16, num_streams=4)
    res, st = srv.run(reqs)
    assert st["completed"] == 12
    assert st["peak_inflight"] <= 2
    assert st["peak_reserved_bytes"] <= 20 << 20
    # the resident plan's tables are charged against the budget
    plan = Q.Plan(20, -1, "unitary", "c64", "bitrev", workspace=False)
    assert st["plan_bytes"] == plan.device_bytes > 0
    assert st["peak_reserved_bytes"] == st["plan_bytes"] + int(res["bytes"][:2].sum())
    plan.close()
    srv.close()
    # a budget the plans alone exceed is refused
    tiny = S.Server(budget_bytes=st["plan_bytes"], max_inflight=4, num_streams=2)
    with pytest.raises(Q.QftError):
        tiny.run(reqs)
    tiny.close()
