"""GPU tests of the autotuner: the tuned configuration is recorded, used by
later plans that ask for it (QFT_PLAN_TUNED) and by no other, and gives
oracle-correct results; batch tuning leaves the per-shape table alone."""

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

def within(y, ref, tol):
    """Relative L2 and max error over the RMS amplitude both <= tol."""
    e = O.error_norms(y, ref)
    return e["rel_l2"] <= tol and e["max_err"] <= tol



@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2606_18981_amd import qft as Q
    assert torch.cuda.is_available()
    Q.tune_clear()
    yield torch, Q
    Q.tune_clear()


def test_tune_shape_and_reuse(env, tmp_path):
    torch, Q = env
    n = 18
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    Q.fill_random(buf, "gaussian", seed=3)
    best, ms = Q.tune(n, -1, "unitary", "c64", "natural", data=buf, reps=2)
    print(f"[gpu] tuned n={n}: {best} {ms:.4f} ms", flush=True)
    assert ms > 0
    assert Q.tune_lookup(n, -1, "c64") == best
    plain = Q.Plan(n, -1, "unitary", "c64", "natural")
    default = Q._cfg_dict(Q.describe(n, -1, "unitary", "c64", "natural").config)
    assert Q._cfg_dict(plain.info.config) == default  # the table is not consulted
    plain.close()
    plan = Q.Plan(n, -1, "unitary", "c64", "natural", tuned=True)
    assert Q._cfg_dict(plan.info.config) == best
    x = I.gaussian(n, 4)
    t = torch.from_numpy(x.astype(np.complex64)).cuda()
    plan.execute(t)
    torch.cuda.synchronize()
    assert within(t.cpu().numpy(), O.qft_fused_targets(x), 1e-5)
    plan.close()
    path = tmp_path / "wisdom.jsonl"
    Q.tune_save(path)
    Q.tune_clear()
    assert Q.tune_load(path) == 1
    assert Q.tune_lookup(n, -1, "c64") == best


def test_tune_batch(env):
    torch, Q = env
    ns, cuts = I.batch_sizes(1004, count=24, lo=8, hi=14, aqft_frac=0.25, aqft_k=8)
    xs = [torch.empty(1 << int(n), dtype=torch.complex64, device="cuda") for n in ns]
    for i, t in enumerate(xs):
        Q.fill_random(t, "uniform", seed=10 + i)
    best, ms = Q.tune_batch(ns.tolist(), cuts.tolist(), xs, reps=1)
    print(f"[gpu] tuned batch: {best} {ms:.4f} ms", flush=True)
    assert ms > 0
    # the per-shape table is not written by batch tuning
    for n, k in zip(ns.tolist(), cuts.tolist()):
        assert Q.tune_lookup(int(n), int(k), "c64") is None
    # the winner, given explicitly, runs the batch with oracle-correct results
    plans = [Q.Plan(int(n), int(k), "unitary", "c64", "natural", config=best)
             for n, k in zip(ns.tolist(), cuts.tolist())]
    hosts = [I.uniform_pm1(int(n), 700 + i) for i, n in enumerate(ns.tolist())]
    ts = [torch.from_numpy(h.astype(np.complex64)).cuda() for h in hosts]
    Q.execute_batch(plans, ts)
    torch.cuda.synchronize()
    for h, t, k in zip(hosts, ts, cuts.tolist()):
        assert within(t.cpu().numpy(), O.qft_fused_targets(h, None if k < 0 else int(k)), 1e-5)
    for p in plans:
        p.close()
    Q.tune_clear()
