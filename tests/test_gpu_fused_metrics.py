"""The accuracy metrics taken in a transform's last pass
(qft_execute_compare, Plan.execute(ref=...)) against the separate
comparison pass (qft_compare, itself checked against the oracle's metric
functions) on the same output and reference, over every kind of last pass:
the generic kernel (tiles smaller than a wave, radix below 32), the
two-group and three-group compile-time kernels, their four-wave forms,
inverse transforms (conjugation on store), bit-reversed output (whose last
pass stores through an exchange-only register group: the generic kernel
takes the comparison there), the AQFT, and the gate schedule.

Bars: the output must equal a plain execute's bit for bit (the comparison
only reads); the sums-based metrics agree with qft_compare's to 1e-12
relative (FP64 sums in another order); the maxima, and the argmax with its
lowest-index tie rule, are identical; a repeated call gives the same bits.
"""

import ctypes
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

SUMS = ("rel_l2", "fidelity", "leakage", "norm_y", "norm_ref", "max_err")


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_18981_amd import qft as Q
    return torch, Q


def tdtype(torch, dtype):
    return torch.complex64 if dtype == "c64" else torch.complex128


def cfg(dtype, split, tiles=None):
    c64 = dtype == "c64"
    c = dict(tile_log2=13 if c64 else 12, radix_log2=5, spec_log2=3 if c64 else 2,
             rev_spec_log2=3 if c64 else 2, pass_bits=split)
    if tiles:
        c["pass_tile_log2"] = tiles
    return c


def same(a, b, rel=1e-12):
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == pytest.approx(b, rel=rel, abs=1e-300)


def check_against_separate(torch, Q, plan, x, ref, what):
    """Run plan on x with and without the fused comparison; compare outputs
    and metrics with qft_compare on the plain output."""
    y_plain = x.clone()
    plan.execute(y_plain)
    y = x.clone()
    mo = torch.full((len(Q.METRIC_NAMES),), -7.0, dtype=torch.float64, device="cuda")
    plan.execute(y, ref=ref, metrics_out=mo)
    torch.cuda.synchronize()
    assert torch.equal(y, y_plain), f"{what}: the compare execute changed the output"
    got = Q.metrics_dict(mo)
    want = Q.compare(y_plain, ref)
    print(f"[fused-metrics] {what}: rel_l2={got['rel_l2']:.3e} fid={got['fidelity']:.15f} "
          f"argmax={got['argmax']}", flush=True)
    for key in SUMS:
        assert same(got[key], want[key]), (what, key, got[key], want[key])
    assert got["argmax"] == want["argmax"], what
    # deterministic
    y2 = x.clone()
    mo2 = torch.empty_like(mo)
    plan.execute(y2, ref=ref, metrics_out=mo2)
    torch.cuda.synchronize()
    assert torch.equal(mo, mo2) or all(
        same(a, b, 0.0) for a, b in zip(mo.cpu().tolist(), mo2.cpu().tolist())), what
    return got


def make_inputs(torch, Q, n, dtype, seed, exact_plan_args):
    """x (Gaussian, on the device) and a reference: the exact transform of x
    under exact_plan_args, perturbed by a small Gaussian term so that the
    difference is not only rounding."""
    x = torch.empty(1 << n, dtype=tdtype(torch, dtype), device="cuda")
    Q.fill_random(x, "gaussian", seed=seed, stream_id=0)
    ref = x.clone()
    ep = Q.Plan(n, -1, *exact_plan_args)
    ep.execute(ref)
    ep.close()
    noise = torch.empty_like(ref)
    Q.fill_random(noise, "gaussian", seed=seed + 1, stream_id=1)
    ref += noise * 1e-4
    return x, ref


# (n, cutoff, dtype, order, inverse, schedule, config, kernel of the last pass)
CASES = [
    (1, -1, "c64", "natural", False, "fused", None, "generic"),
    (4, 1, "c128", "bitrev", False, "fused", None, "generic"),
    (7, -1, "c64", "natural", True, "fused", None, "generic"),
    (12, 4, "c64", "natural", False, "fused", dict(tile_log2=10, radix_log2=3), "generic"),
    (13, -1, "c128", "bitrev", False, "fused", dict(tile_log2=9, radix_log2=4), "generic"),
    (16, 6, "c64", "natural", False, "fused", None, "two"),
    (16, -1, "c128", "natural", True, "fused", None, "two"),
    (16, -1, "c128", "bitrev", True, "fused", None, "two-x"),
    (20, 5, "c64", "bitrev", False, "fused", None, "two-x"),
    (20, -1, "c64", "natural", True, "fused", None, "two"),
    (24, 8, "c64", "natural", False, "fused", cfg("c64", [7, 6, 11]), "three"),
    (24, -1, "c64", "natural", True, "fused", cfg("c64", [7, 6, 11]), "three"),
    (24, -1, "c64", "bitrev", True, "fused", cfg("c64", [7, 6, 11]), "generic"),
    (22, -1, "c128", "natural", False, "fused", cfg("c128", [6, 5, 11]), "three"),
    (24, -1, "c64", "natural", False, "fused", cfg("c64", [6, 10, 8], [14, 14, 14]), "two-lean"),
    (24, 6, "c64", "natural", True, "fused", cfg("c64", [6, 7, 11], [13, 14, 14]), "three-lean"),
    (24, -1, "c128", "natural", True, "fused", cfg("c128", [6, 10, 8], [13, 13, 13]),
     "two-lean"),
    (12, 3, "c64", "natural", False, "gates", None, "gates"),
]


def last_kernel_kind(Q, plan, dtype, config):
    info = plan.info
    if info.layout & Q.QFT_SCHEDULE_GATES:
        return "gates"
    kern = info.pass_kernel[info.num_passes - 1]
    if kern == 0:
        return "generic"
    if kern >= 17:
        return "two-x"  # with the store exchange (a bit-reversed-order last pass)
    kind = "three" if kern > 10 else "two"
    tiles = (config or {}).get("pass_tile_log2")
    if tiles and tiles[-1] == (14 if dtype == "c64" else 13):
        kind += "-lean"
    return kind


@pytest.mark.parametrize("n,k,dtype,order,inverse,schedule,config,kind", CASES)
def test_fused_metrics_match_separate(env, n, k, dtype, order, inverse, schedule, config, kind):
    torch, Q = env
    what = f"n={n} k={k} {dtype} {order} inverse={inverse} {schedule} {config} ({kind})"
    print(f"[gpu] {what}", flush=True)
    plan = Q.Plan(n, k, "unitary", dtype, order, schedule, config, inverse=inverse)
    assert last_kernel_kind(Q, plan, dtype, config) == kind
    x, ref = make_inputs(torch, Q, n, dtype, 9100 + n,
                         ("unitary", dtype, order, "fused", None, True, inverse))
    check_against_separate(torch, Q, plan, x, ref, what)
    plan.close()


@pytest.mark.parametrize("n,dtype,order", [(28, "c64", "natural"), (26, "c128", "natural"),
                                           (28, "c64", "bitrev")])
def test_fused_metrics_default_plans_large(env, n, dtype, order):
    # the default plans of the headline sizes, AQFT against the exact
    # transform: the measured error sits at the closed-form expectation
    torch, Q = env
    k = 10
    print(f"[gpu] fused metrics default plan n={n} {dtype} {order} k={k}", flush=True)
    x = torch.empty(1 << n, dtype=tdtype(torch, dtype), device="cuda")
    Q.fill_random(x, "gaussian", seed=9200 + n, stream_id=0)
    ref = x.clone()
    ep = Q.Plan(n, -1, "unitary", dtype, order)
    ep.execute(ref)
    ep.close()
    plan = Q.Plan(n, k, "unitary", dtype, order)
    got = check_against_separate(torch, Q, plan, x, ref, f"default n={n} {dtype} {order} k={k}")
    assert got["rel_l2"] == pytest.approx(Q.expected_error(n, k), rel=0.05)
    plan.close()
    del x, ref
    torch.cuda.empty_cache()


def test_fused_metrics_oracle_small(env):
    # one case checked directly against the oracle's metric functions
    torch, Q = env
    n, k = 10, 3
    x = I.gaussian(n, 9300)
    t = torch.from_numpy(x.astype(np.complex128)).cuda()
    ref_np = O.qft_fused_targets(x, None)
    ref = torch.from_numpy(ref_np).cuda()
    plan = Q.Plan(n, k, "unitary", "c128", "natural")
    mo = torch.empty(len(Q.METRIC_NAMES), dtype=torch.float64, device="cuda")
    plan.execute(t, ref=ref, metrics_out=mo)
    got = Q.metrics_dict(mo)
    y = t.cpu().numpy()
    want = {"rel_l2": O.rel_l2(y, ref_np), "max_err": O.max_err(y, ref_np),
            "fidelity": O.fidelity(y, ref_np), "leakage": O.top_bin_leakage(y, ref_np),
            "norm_y": float(np.linalg.norm(y)), "norm_ref": float(np.linalg.norm(ref_np))}
    for key, v in want.items():
        assert got[key] == pytest.approx(v, rel=1e-9, abs=1e-12), key
    assert got["argmax"] == int(np.argmax(np.abs(ref_np)))
    plan.close()


def test_fused_metrics_ties_and_zero_reference(env):
    torch, Q = env
    n = 18
    for dtype in ("c64", "c128"):
        plan = Q.Plan(n, 5, "unitary", dtype, "natural")
        x = torch.empty(1 << n, dtype=tdtype(torch, dtype), device="cuda")
        Q.fill_random(x, "gaussian", seed=9400, stream_id=0)
        # a zero reference: every |r|^2 ties at 0, so the argmax is index 0
        zero = torch.zeros_like(x)
        got = check_against_separate(torch, Q, plan, x, zero, f"zero reference {dtype}")
        assert got["argmax"] == 0 and got["norm_ref"] == 0.0
        # equal maxima at several indices: the lowest one wins
        for a, b in ((5, 1 << 17), (1 << 12, (1 << 12) + 1), (777, 778 + (1 << 10))):
            ref = torch.zeros_like(x)
            Q.fill_random(ref, "uniform", seed=9401, stream_id=0)
            ref[b] = 40.0
            ref[a] = 40.0
            got = check_against_separate(torch, Q, plan, x, ref, f"tie {a},{b} {dtype}")
            assert got["argmax"] == a
        plan.close()


def test_fused_metrics_errors(env):
    torch, Q = env
    n = 12
    plan = Q.Plan(n, -1, "unitary", "c64", "natural")
    x = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    mo = torch.empty(len(Q.METRIC_NAMES), dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QftError):
        plan.execute(x, ref=x, metrics_out=mo)  # the reference overlaps the data
    # ... or the workspace the earlier passes of a multi-pass plan write
    p16 = Q.Plan(16, -1, "unitary", "c64", "natural")
    x16 = torch.zeros(1 << 16, dtype=torch.complex64, device="cuda")
    ws = torch.empty(p16.info.workspace_bytes // 8, dtype=torch.complex64, device="cuda")
    assert ws.numel() == x16.numel()
    with pytest.raises(Q.QftError):
        p16.execute(x16, workspace=ws, ref=ws, metrics_out=mo)
    p16.close()
    with pytest.raises(ValueError):
        plan.execute(x, ref=x.clone(), metrics_out=mo.float())
    with pytest.raises(ValueError):
        plan.execute(x, metrics_out=mo)
    ws = torch.empty(max(1, plan.compare_workspace_bytes() // 8), dtype=torch.float64,
                     device="cuda")
    rc = Q.lib.qft_execute_compare(plan.handle, ctypes.c_void_p(x.data_ptr()), None, None,
                                   ctypes.c_void_p(ws.data_ptr()),
                                   ctypes.c_void_p(mo.data_ptr()), None)
    assert rc == Q.QFT_ERR_POINTER
    assert Q.lib.qft_execute_compare_workspace_bytes(None) == 0
    plan.close()
