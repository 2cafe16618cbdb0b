"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances against the oracle, both asserted on every comparison: relative
L2 and max error over the RMS amplitude (oracle.error_norms), each <= 1e-12
for complex128 and <= 1e-5 for complex64, at every n tested here.  The
max-error bar is the stronger one (max error >= relative L2 always), so a
single wrong element fails it.  Inputs are seeded synthetic arrays from
paper_2606_18981_amd.inputs.
"""

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def Q():
    from paper_2606_18981_amd import qft
    return qft


def run_gpu(torch, Q, x, n, cutoff=-1, norm="unitary", dtype="c64", order="natural",
            schedule="fused", config=None, inverse=False):
    print(f"[gpu] n={n} cutoff={cutoff} norm={norm} dtype={dtype} order={order} "
          f"schedule={schedule} config={config} inverse={inverse}", flush=True)
    plan = Q.Plan(n, cutoff, norm, dtype, order, schedule, config, inverse=inverse)
    t = torch.from_numpy(np.asarray(x).astype(NPDT[dtype])).to("cuda")
    plan.execute(t)
    torch.cuda.synchronize()
    y = t.cpu().numpy().astype(np.complex128)
    plan.close()
    return y


def close(y, ref, dtype):
    """Relative L2 and max error over the RMS amplitude, both within the
    element type's bar."""
    e = O.error_norms(y, ref)
    return e["rel_l2"] <= TOL[dtype] and e["max_err"] <= TOL[dtype]


def oracle_ref(x, cutoff, norm, order, inverse=False):
    n = int(np.log2(len(x)))
    k = None if cutoff < 0 else cutoff
    if n <= 11:
        return O.qft_circuit(x, k, norm, order, inverse=inverse)
    return O.qft_fused_targets(x, k, norm, order, inverse=inverse)


# ---- config 1: plain exact n = 10, complex128, gate by gate ---------------

@pytest.mark.parametrize("schedule", ["gates", "fused"])
@pytest.mark.parametrize("which", ["uniform", "delta", "tone37"])
def test_n10_c128_three_inputs(torch_cuda, Q, schedule, which):
    n = 10
    x = {"uniform": I.uniform_pm1(n, 1001), "delta": I.delta(n, 0),
         "tone37": I.tone(n, 37)}[which]
    y = run_gpu(torch_cuda, Q, x, n, -1, "unitary", "c128", "natural", schedule)
    ref = O.dft_naive(x)
    assert close(y, ref, "c128")
    if which == "delta":
        assert np.max(np.abs(y - 1.0 / 32)) < 1e-14
    if which == "tone37":
        spike = np.zeros(1 << n, complex)
        spike[37] = 32.0
        assert np.max(np.abs(y - spike)) < 1e-12


# ---- sweep of sizes, dtypes, orders and norms -------------------------------

SWEEP = []
for n in list(range(1, 21)):
    for dt in ("c64", "c128"):
        SWEEP.append((n, dt, "natural", "unitary"))
for n in (3, 12, 13, 14, 17):
    for dt in ("c64", "c128"):
        SWEEP.append((n, dt, "bitrev", "unitary"))
        SWEEP.append((n, dt, "natural", "none"))
        SWEEP.append((n, dt, "bitrev", "inv_n"))


@pytest.mark.parametrize("n,dtype,order,norm", SWEEP)
def test_exact_sweep(torch_cuda, Q, n, dtype, order, norm):
    x = I.gaussian(n, 2000 + n)
    y = run_gpu(torch_cuda, Q, x, n, -1, norm, dtype, order)
    assert close(y, oracle_ref(x, -1, norm, order), dtype)


@pytest.mark.parametrize("n", [4, 9, 12, 16, 20])
@pytest.mark.parametrize("k", [0, 1, 2, 3, 6, 10])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_aqft_sweep(torch_cuda, Q, n, k, dtype):
    x = I.gaussian(n, 3000 + n)
    y = run_gpu(torch_cuda, Q, x, n, k, "unitary", dtype, "natural")
    assert close(y, oracle_ref(x, k, "unitary", "natural"), dtype)


CONFIGS = [
    dict(tile_log2=6, radix_log2=1, spec_log2=2, rev_spec_log2=2),
    dict(tile_log2=8, radix_log2=3, spec_log2=-1, rev_spec_log2=-1),
    dict(tile_log2=9, radix_log2=5, spec_log2=4, rev_spec_log2=4),
    dict(tile_log2=12, radix_log2=4, spec_log2=4, rev_spec_log2=4),
    dict(tile_log2=13, radix_log2=5, spec_log2=3, rev_spec_log2=3),
    dict(tile_log2=12, radix_log2=5, spec_log2=2, rev_spec_log2=2),
    dict(tile_log2=11, radix_log2=3, spec_log2=2, rev_spec_log2=2),
    dict(tile_log2=14, radix_log2=5, spec_log2=4, rev_spec_log2=4),
    dict(tile_log2=12, radix_log2=4, spec_log2=2, rev_spec_log2=3, pass_bits=[7, 7, 6]),
    # streaming (non-temporal) access on every pass that reads whole lines
    dict(tile_log2=13, radix_log2=5, spec_log2=3, rev_spec_log2=3, nontemporal=2),
    dict(tile_log2=11, radix_log2=5, spec_log2=4, rev_spec_log2=4, nontemporal=2),
]


@pytest.mark.parametrize("cfg", CONFIGS)
@pytest.mark.parametrize("n,k,order", [(11, -1, "natural"), (19, 4, "natural"),
                                       (20, -1, "bitrev"), (20, 6, "natural")])
def test_kernel_configs(torch_cuda, Q, cfg, n, k, order):
    if "pass_bits" in cfg and sum(cfg["pass_bits"]) != n:
        pytest.skip("explicit split is for n = 20")
    for dt in ("c64", "c128"):
        x = I.uniform_pm1(n, 4000 + n)
        y = run_gpu(torch_cuda, Q, x, n, k, "unitary", dt, order, "fused", cfg)
        assert close(y, oracle_ref(x, k, "unitary", order), dt)


def test_gate_schedule_matches_fused_on_gpu(torch_cuda, Q):
    n = 12
    x = I.gaussian(n, 5)
    for k in (-1, 3):
        a = run_gpu(torch_cuda, Q, x, n, k, "unitary", "c128", "natural", "gates")
        b = run_gpu(torch_cuda, Q, x, n, k, "unitary", "c128", "natural", "fused")
        assert O.rel_l2(a, b) <= 1e-13
        assert close(a, oracle_ref(x, k, "unitary", "natural"), "c128")


# ---- config 2: n = 24, both dtypes, Gaussian and multi-tone ----------------

@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_n24_gaussian_and_tones(torch_cuda, Q, dtype):
    n = 24
    x = I.gaussian(n, 1002, unit_norm=True)
    y = run_gpu(torch_cuda, Q, x, n, -1, "unitary", dtype, "natural")
    ref = O.qft_fused_targets(x)
    assert close(y, ref, dtype)
    xt, bins, amp, ph = I.multi_tone(n, 1002, 8, 0.01)
    y = run_gpu(torch_cuda, Q, xt, n, -1, "unitary", dtype, "natural")
    sample = np.concatenate([bins, np.random.default_rng(1).choice(1 << n, 24, replace=False)])
    assert close(y[sample], O.dft_bins(xt, sample), dtype)
    assert np.linalg.norm(y) == pytest.approx(np.linalg.norm(xt), rel=1e-5)
    for b, a, p in zip(bins, amp, ph):
        assert abs(y[b] - a * np.exp(1j * p) * 2 ** (n / 2)) < 1.0


# ---- config 3 at full size: tests/test_gpu_full_parity.py (whole vector) --

@pytest.mark.timeout(900)
def test_n31_maximum_size(torch_cuda, Q):
    """The largest supported transform, 2^31 complex64 elements (16 GiB, a
    four-pass plan), exact and AQFT, on sampled bins, and Parseval."""
    torch = torch_cuda
    n = 31
    print("[gpu] n=31 input", flush=True)
    x = I.gaussian(n, 3100)
    bins = np.random.default_rng(31).choice(1 << n, 12, replace=False)
    nx = float(np.sqrt(np.vdot(x, x).real))
    print("[gpu] n=31 oracle bins", flush=True)
    refs = {-1: O.dft_bins(x, bins), 10: O.aqft_bins(x, bins, 10)}
    xd = torch.from_numpy(x.astype(np.complex64)).cuda()
    del x
    bd = torch.from_numpy(bins).cuda()
    for k in (-1, 10):
        print(f"[gpu] n=31 cutoff={k}", flush=True)
        plan = Q.Plan(n, k, "unitary", "c64", "natural")
        assert plan.info.num_passes == 4
        t = xd.clone()
        plan.execute(t)
        torch.cuda.synchronize()
        y = t[bd].cpu().numpy().astype(np.complex128)
        ny = float(torch.sqrt((t.real.double() ** 2).sum() + (t.imag.double() ** 2).sum()))
        del t
        plan.close()
        assert close(y, refs[k], "c64")
        assert ny == pytest.approx(nx, rel=1e-5)
    del xd
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
@pytest.mark.timeout(600)
def test_n30_c128_whole_vector(torch_cuda, Q):
    """complex128 at n = 30 (16 GiB): the default three-pass plan (2^13 lean
    tiles) and an explicit four-pass split with 2^12 tiles, every output
    element against the oracle's whole-vector form (plain C, FP64), the
    AQFT on sampled bins, and Parseval."""
    torch = torch_cuda
    n = 30
    print("[gpu] n=30 c128 input", flush=True)
    x = I.gaussian(n, 3000)
    bins = np.random.default_rng(30).choice(1 << n, 12, replace=False)
    nx = float(np.sqrt(np.vdot(x, x).real))
    print("[gpu] n=30 c128 oracle, whole vector", flush=True)
    ref = O.qft_state_c(x, None)
    ref9 = O.aqft_bins(x, bins, 9)
    xd = torch.from_numpy(x).cuda()
    del x
    four = dict(tile_log2=12, radix_log2=5, spec_log2=2, rev_spec_log2=2,
                pass_bits=[6, 8, 8, 8], pass_tile_log2=[12, 12, 12, 12])
    for what, k, cfg, P in (("default", -1, None, 3), ("four-pass", -1, four, 4),
                            ("default", 9, None, 3)):
        print(f"[gpu] n=30 c128 {what} cutoff={k}", flush=True)
        plan = Q.Plan(n, k, "unitary", "c128", "natural", config=cfg)
        assert plan.info.num_passes == P
        t = xd.clone()
        plan.execute(t)
        torch.cuda.synchronize()
        ny = float(torch.linalg.vector_norm(t))
        plan.close()
        if k < 0:
            y = t.cpu().numpy()
            del t
            e = O.error_norms(y, ref)
            print(f"[parity] n=30 c128 {what}: rel_l2={e['rel_l2']:.3e} "
                  f"max_err={e['max_err']:.3e}", flush=True)
            assert e["rel_l2"] <= TOL["c128"] and e["max_err"] <= TOL["c128"]
            del y
        else:
            y = t[torch.from_numpy(bins).cuda()].cpu().numpy()
            del t
            assert close(y, ref9, "c128")
        assert ny == pytest.approx(nx, rel=1e-12)
    del xd, ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [-1, 5])
def test_wide_first_pass_plan(torch_cuda, Q, k):
    """The first pass with one more tile bit than the others (2^11 against
    2^10), the rule that n = 30 takes at the default tiles."""
    n = 21
    cfg = dict(tile_log2=10, radix_log2=4, spec_log2=3, rev_spec_log2=3)
    x = I.gaussian(n, 2100)
    y = run_gpu(torch_cuda, Q, x, n, k, "unitary", "c64", "natural", "fused", cfg)
    assert close(y, O.qft_fused_targets(x, None if k < 0 else k), "c64")


# ---- inverse (conjugate-phase) transform ----------------------------------

INV = []
for n in (1, 5, 10, 13, 14, 20):
    for dt in ("c64", "c128"):
        INV.append((n, -1, dt, "natural", "unitary", "fused"))
INV += [(12, 3, "c64", "bitrev", "none", "fused"), (18, 6, "c128", "natural", "inv_n", "fused"),
        (9, -1, "c128", "natural", "unitary", "gates"), (11, 4, "c64", "bitrev", "inv_n", "gates")]


@pytest.mark.parametrize("n,k,dtype,order,norm,schedule", INV)
def test_inverse_sweep(torch_cuda, Q, n, k, dtype, order, norm, schedule):
    x = I.gaussian(n, 6000 + n)
    y = run_gpu(torch_cuda, Q, x, n, k, norm, dtype, order, schedule, inverse=True)
    assert close(y, oracle_ref(x, k, norm, order, inverse=True), dtype)


@pytest.mark.parametrize("cfg", [CONFIGS[4], CONFIGS[5], CONFIGS[8]])
def test_inverse_kernel_configs(torch_cuda, Q, cfg):
    n = 20
    for dt in ("c64", "c128"):
        x = I.uniform_pm1(n, 6100)
        y = run_gpu(torch_cuda, Q, x, n, 5, "unitary", dt, "natural", "fused", cfg, inverse=True)
        assert close(y, oracle_ref(x, 5, "unitary", "natural", inverse=True), dt)


@pytest.mark.parametrize("k", [-1, 7])
def test_forward_then_inverse_is_identity(torch_cuda, Q, k):
    torch = torch_cuda
    n = 22
    x = I.gaussian(n, 6200)
    t = torch.from_numpy(x).cuda()
    fwd = Q.Plan(n, k, "unitary", "c128", "natural")
    inv = Q.Plan(n, k, "unitary", "c128", "natural", inverse=True)
    fwd.execute(t)
    inv.execute(t)
    torch.cuda.synchronize()
    assert close(t.cpu().numpy(), x, "c128")
    fwd.close()
    inv.close()


# ---- input norm as metadata (the paper's scale_in) -------------------------

@pytest.mark.parametrize("n,dtype,schedule", [(1, "c64", "fused"), (5, "c128", "fused"),
                                              (10, "c64", "gates"), (12, "c128", "gates"),
                                              (13, "c64", "fused"), (20, "c128", "fused"),
                                              (24, "c64", "fused")])
def test_execute_norm(torch_cuda, Q, n, dtype, schedule):
    torch = torch_cuda
    import ctypes
    print(f"[gpu] norm n={n} dtype={dtype} schedule={schedule}", flush=True)
    x = (I.gaussian(n, 6300 + n) * 3.7).astype(NPDT[dtype])
    plan = Q.Plan(n, -1, "unitary", dtype, "natural", schedule)
    a = torch.from_numpy(x).cuda()
    b = a.clone()
    norm = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    plan.execute(a)
    plan.execute(b, norm_out=norm)
    plan.execute(b.clone(), norm_out=norm)  # a second call reuses the partial sums
    torch.cuda.synchronize()
    assert torch.equal(a, b), "the norm must not change the transform"
    ref = float(np.linalg.norm(x.astype(np.complex128)))
    got = float(norm.cpu()[0])
    assert abs(got - ref) <= (1e-13 if dtype == "c128" else 1e-6) * ref
    rc = Q.lib.qft_execute_norm(plan.handle, ctypes.c_void_p(b.data_ptr()), None, None, None)
    assert rc == Q.QFT_ERR_POINTER
    plan.close()


# ---- lengths that are not powers of two --------------------------------------

@pytest.mark.parametrize("N,dtype", [(3, "c64"), (1000, "c128"), (70000, "c64"), (1, "c128")])
def test_padded_transform(torch_cuda, Q, N, dtype):
    torch = torch_cuda
    import ctypes
    print(f"[gpu] padded N={N} {dtype}", flush=True)
    rng = np.random.default_rng(N)
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(NPDT[dtype])
    t = Q.padded(torch.from_numpy(x).cuda())
    M = t.numel()
    assert M == max(2, 1 << (N - 1).bit_length())
    host = t.cpu().numpy()
    assert np.array_equal(host[:N], x) and not np.any(host[N:])
    n = M.bit_length() - 1
    plan = Q.Plan(n, -1, "unitary", dtype, "natural")
    plan.execute(t)
    torch.cuda.synchronize()
    ref = O.qft_padded(x.astype(np.complex128)) if N > 1 else O.qft_circuit(
        np.array([x[0], 0], dtype=np.complex128))
    assert close(t.cpu().numpy().astype(np.complex128), ref, dtype)
    plan.close()
    # overlapping buffers are refused
    rc = Q.lib.qft_pad(ctypes.c_void_p(t.data_ptr()), 1, ctypes.c_void_p(t.data_ptr()), n,
                       Q.layout_flags(dtype), None)
    assert rc == Q.QFT_ERR_INVALID


# ---- device input generator ------------------------------------------------

@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_device_philox_matches_host(torch_cuda, Q, dtype):
    torch = torch_cuda
    n = 16
    t = torch.empty(1 << n, dtype=torch.complex128 if dtype == "c128" else torch.complex64,
                    device="cuda")
    Q.fill_random(t, "uniform", seed=1234, stream_id=7)
    torch.cuda.synchronize()
    host = I.philox_uniform_pm1(n, 1234, 7).astype(NPDT[dtype])
    assert np.array_equal(t.cpu().numpy(), host)
    Q.fill_random(t, "gaussian", seed=99, stream_id=3)
    torch.cuda.synchronize()
    host = I.philox_gaussian(n, 99, 3)
    got = t.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - host)) <= (1e-13 if dtype == "c128" else 1e-6)


# ---- ABI behaviour on the device ------------------------------------------

def test_abi_errors_and_workspace(torch_cuda, Q):
    torch = torch_cuda
    import ctypes
    n = 18
    plan = Q.Plan(n, -1, "unitary", "c64", "natural")
    t = torch.zeros((1 << n) + 1, dtype=torch.complex64, device="cuda")
    # misaligned pointer -> QFT_ERR_POINTER, nothing launched
    rc = Q.lib.qft_execute(plan.handle, ctypes.c_void_p(t.data_ptr() + 4), None)
    assert rc == Q.QFT_ERR_POINTER
    rc = Q.lib.qft_execute(plan.handle, None, None)
    assert rc == Q.QFT_ERR_POINTER
    rc = Q.lib.qft_execute_ws(plan.handle, ctypes.c_void_p(t.data_ptr()), None, None)
    assert rc == Q.QFT_ERR_POINTER  # this plan needs a workspace
    # caller workspaces on two streams give the plan's own result
    x = I.gaussian(n, 9)
    a = torch.from_numpy(x.astype(np.complex64)).cuda()
    b = a.clone()
    c = a.clone()
    ws1 = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    ws2 = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.execute(a)
    plan.execute(b, stream=s1, workspace=ws1)
    plan.execute(c, stream=s2, workspace=ws2)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    # device memory the plan holds: tables + its own workspace
    info = plan.info
    assert plan.device_bytes == info.table_bytes + info.workspace_bytes
    bare = Q.Plan(n, -1, "unitary", "c64", "natural", workspace=False)
    assert bare.device_bytes == bare.info.table_bytes
    bare.close()
    assert Q.lib.qft_plan_device_bytes(None) == 0
    plan.close()


def test_timing_api(torch_cuda, Q):
    torch = torch_cuda
    n = 22
    plan = Q.Plan(n, -1, "unitary", "c64", "natural")
    t = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    Q.fill_random(t, "gaussian", seed=1)
    plan.set_timing(True)
    for _ in range(3):
        plan.execute(t)
    ms, ex = plan.pass_times()
    assert ex == 3
    assert len(ms) == plan.info.num_passes and all(m > 0 for m in ms)
    plan.close()
