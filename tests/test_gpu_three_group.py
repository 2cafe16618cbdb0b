"""GPU parity of the three-group pass kernel (passes of 11-13 qubits whose
last register group is reached by cross-lane swaps) against the FP64
oracle, on the whole output vector.

Explicit pass splits place such a pass first (below-pass diagonal, input
norm, inverse conjugation on load), in the middle, and last (bit-reversed
stores, conjugation on store), in complex64 (2^13-element tiles) and
complex128 (2^12).  Bars as everywhere: relative L2 and max error over the
RMS amplitude, each <= 1e-5 (complex64) or <= 1e-12 (complex128).  Batched
runs of the same plans must equal the lone runs bit for bit.
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


def cfg(dtype, split, **kw):
    c64 = dtype == "c64"
    c = dict(tile_log2=13 if c64 else 12, radix_log2=5, spec_log2=3 if c64 else 2,
             rev_spec_log2=3 if c64 else 2, pass_bits=split)
    c.update(kw)
    return c


def check(y, ref, dtype, what):
    e = O.error_norms(y, ref)
    print(f"[parity] {what}: rel_l2={e['rel_l2']:.3e} max_err={e['max_err']:.3e}", flush=True)
    assert e["rel_l2"] <= TOL[dtype] and e["max_err"] <= TOL[dtype], (what, e)


def run(torch, Q, x, n, k, norm, dtype, order, config, inverse=False, norm_out=False,
        three=True):
    print(f"[gpu] n={n} k={k} norm={norm} {dtype} {order} {config} inverse={inverse}",
          flush=True)
    plan = Q.Plan(n, k, norm, dtype, order, "fused", config, inverse=inverse)
    if three:
        assert any(11 <= plan.info.pass_kernel[p] <= 16 for p in range(plan.info.num_passes))
    t = torch.from_numpy(x.astype(NPDT[dtype])).cuda()
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda") if norm_out else None
    plan.execute(t, norm_out=nrm)
    torch.cuda.synchronize()
    y = t.cpu().numpy().astype(np.complex128)
    plan.close()
    return (y, float(nrm.item())) if norm_out else y


SPLITS = [
    ("c64", [6, 11, 7]), ("c64", [5, 12, 7]), ("c64", [4, 13, 7]), ("c64", [11, 6, 7]),
    ("c64", [7, 6, 11]), ("c64", [11, 13]), ("c128", [5, 11, 6]), ("c128", [5, 12, 5]),
    ("c128", [6, 5, 11]),
]


@pytest.mark.parametrize("dtype,split", SPLITS)
def test_three_group_splits(torch_cuda, Q, dtype, split):
    n = sum(split)
    x = I.gaussian(n, 5100 + n)
    c = cfg(dtype, split)
    for k, order, norm in ((-1, "natural", "unitary"), (6, "natural", "unitary"),
                           (10, "bitrev", "none")):
        # a last pass of a bit-reversed-order plan stores through one more
        # exchange (lowest global bits back on the lanes): the generic kernel
        three = not (order == "bitrev" and split[-1] > 10 and len(split) == 3)
        y = run(torch_cuda, Q, x, n, k, norm, dtype, order, c, three=three)
        ref = O.qft_fused_targets(x, None if k < 0 else k, norm, order)
        check(y, ref, dtype, f"n={n} {split} k={k} {order} {norm}")


@pytest.mark.parametrize("dtype,split", [("c64", [11, 6, 7]), ("c64", [5, 12, 7]),
                                         ("c128", [6, 5, 11])])
def test_three_group_inverse_and_norm(torch_cuda, Q, dtype, split):
    n = sum(split)
    x = I.gaussian(n, 5200 + n) * 3.0
    c = cfg(dtype, split)
    y = run(torch_cuda, Q, x, n, -1, "inv_n", dtype, "natural", c, inverse=True)
    check(y, O.qft_fused_targets(x, None, "inv_n", "natural", inverse=True), dtype,
          f"inverse n={n} {split}")
    y, nrm = run(torch_cuda, Q, x, n, 8, "unitary", dtype, "natural", c, norm_out=True)
    check(y, O.qft_fused_targets(x, 8), dtype, f"norm n={n} {split}")
    assert nrm == pytest.approx(float(np.linalg.norm(x)), rel=1e-6 if dtype == "c64" else 1e-12)


def test_three_group_streaming(torch_cuda, Q):
    # non-temporal loads and stores on a three-group pass that reads whole
    # lines: the bit-reversing last pass loads 2^11-element contiguous runs
    n = 24
    x = I.gaussian(n, 5300)
    for dtype, split in (("c64", [7, 6, 11]), ("c128", [7, 6, 11])):
        c = cfg(dtype, split, nontemporal=2)
        info = Q.describe(n, -1, "unitary", dtype, "natural", "fused", c)
        assert 11 <= info.pass_kernel[2] <= 16 and info.pass_streaming[2] == 1
        y = run(torch_cuda, Q, x, n, -1, "unitary", dtype, "natural", c)
        check(y, O.qft_fused_targets(x, None), dtype, f"streaming {dtype} {split}")


def test_three_group_batch_bitwise(torch_cuda, Q):
    torch = torch_cuda
    specs = [(20, -1, [4, 11, 5]), (21, 8, [4, 12, 5]), (22, -1, [4, 13, 5]),
             (20, 6, [5, 4, 11]), (18, -1, [7, 11])]
    plans, xs, alone = [], [], []
    for i, (n, k, split) in enumerate(specs):
        p = Q.Plan(n, k, "unitary", "c64", "natural", "fused", cfg("c64", split))
        plans.append(p)
        x = I.uniform_pm1(n, 5400 + i)
        t = torch.from_numpy(x.astype(np.complex64)).cuda()
        xs.append(t)
        a = t.clone()
        p.execute(a)
        alone.append(a)
    print("[gpu] batch of three-group plans", flush=True)
    Q.execute_batch(plans, xs, graph=True)
    torch.cuda.synchronize()
    for (n, k, split), t, a in zip(specs, xs, alone):
        assert torch.equal(t, a), f"batched n={n} {split} differs from the lone run"
    for p in plans:
        p.close()


# ---- the four-wave forms: 2^14-element complex64 tiles of 512 threads ------

WIDE = [
    ([6, 10, 6], [14, 14, 13]), ([7, 11, 6], [14, 14, 13]), ([6, 10, 8], [14, 14, 14]),
    ([5, 12, 7], [13, 14, 14]),
]


@pytest.mark.parametrize("split,tiles", WIDE)
def test_four_wave_wide_tiles(torch_cuda, Q, split, tiles):
    n = sum(split)
    x = I.gaussian(n, 5500 + n)
    c = cfg("c64", split, pass_tile_log2=tiles)
    info = Q.describe(n, -1, "unitary", "c64", "natural", "fused", c)
    for p, t in enumerate(tiles):
        assert info.pass_spec[p] == t - split[p]
    for k, order, norm in ((-1, "natural", "unitary"), (6, "bitrev", "inv_n")):
        y = run(torch_cuda, Q, x, n, k, norm, "c64", order, c, three=False)
        ref = O.qft_fused_targets(x, None if k < 0 else k, norm, order)
        check(y, ref, "c64", f"wide n={n} {split} {tiles} k={k} {order}")
    y = run(torch_cuda, Q, x, n, -1, "none", "c64", "natural", c, inverse=True, three=False)
    check(y, O.qft_fused_targets(x, None, "none", "natural", inverse=True), "c64",
          f"wide inverse n={n} {split}")
    y, nrm = run(torch_cuda, Q, x, n, 8, "unitary", "c64", "natural", c, norm_out=True,
                 three=False)
    check(y, O.qft_fused_targets(x, 8), "c64", f"wide norm n={n} {split}")
    assert nrm == pytest.approx(float(np.linalg.norm(x)), rel=1e-6)


def test_four_wave_batch_bitwise(torch_cuda, Q):
    torch = torch_cuda
    specs = [(20, -1, [5, 10, 5], [14, 14, 13]), (21, 8, [5, 11, 5], [14, 14, 14]),
             (22, -1, [6, 10, 6], [14, 13, 14])]
    plans, xs, alone = [], [], []
    for i, (n, k, split, tiles) in enumerate(specs):
        p = Q.Plan(n, k, "unitary", "c64", "natural", "fused",
                   cfg("c64", split, pass_tile_log2=tiles))
        plans.append(p)
        t = torch.from_numpy(I.uniform_pm1(n, 5600 + i).astype(np.complex64)).cuda()
        xs.append(t)
        a = t.clone()
        p.execute(a)
        alone.append(a)
    print("[gpu] batch of four-wave plans", flush=True)
    Q.execute_batch(plans, xs, graph=True)
    torch.cuda.synchronize()
    for (n, k, split, tiles), t, a in zip(specs, xs, alone):
        assert torch.equal(t, a), f"batched n={n} {split} {tiles} differs from the lone run"
    for p in plans:
        p.close()


# ---- the lean complex128 forms: 2^13-element tiles of 256 threads ---------

WIDE128 = [([6, 10, 6], [13, 13, 12]), ([5, 11, 6], [13, 13, 12]), ([6, 10, 8], [13, 13, 13])]


@pytest.mark.parametrize("split,tiles", WIDE128)
def test_lean_c128_wide_tiles(torch_cuda, Q, split, tiles):
    n = sum(split)
    x = I.gaussian(n, 5700 + n)
    c = cfg("c128", split, pass_tile_log2=tiles)
    info = Q.describe(n, -1, "unitary", "c128", "natural", "fused", c)
    for p, t in enumerate(tiles):
        assert info.pass_spec[p] == t - split[p]
    for k, order, norm in ((-1, "natural", "unitary"), (6, "bitrev", "inv_n")):
        y = run(torch_cuda, Q, x, n, k, norm, "c128", order, c, three=False)
        ref = O.qft_fused_targets(x, None if k < 0 else k, norm, order)
        check(y, ref, "c128", f"lean c128 n={n} {split} {tiles} k={k} {order}")
    y = run(torch_cuda, Q, x, n, -1, "none", "c128", "natural", c, inverse=True, three=False)
    check(y, O.qft_fused_targets(x, None, "none", "natural", inverse=True), "c128",
          f"lean c128 inverse n={n} {split}")


def test_lean_c128_batch_bitwise(torch_cuda, Q):
    torch = torch_cuda
    specs = [(20, -1, [5, 10, 5], [13, 13, 12]), (21, 8, [5, 11, 5], [13, 13, 12]),
             (22, -1, [6, 10, 6], [13, 12, 13])]
    plans, xs, alone = [], [], []
    for i, (n, k, split, tiles) in enumerate(specs):
        p = Q.Plan(n, k, "unitary", "c128", "natural", "fused",
                   cfg("c128", split, pass_tile_log2=tiles))
        plans.append(p)
        t = torch.from_numpy(I.uniform_pm1(n, 5800 + i)).cuda()
        xs.append(t)
        a = t.clone()
        p.execute(a)
        alone.append(a)
    print("[gpu] batch of lean complex128 plans", flush=True)
    Q.execute_batch(plans, xs, graph=True)
    torch.cuda.synchronize()
    for (n, k, split, tiles), t, a in zip(specs, xs, alone):
        assert torch.equal(t, a), f"batched n={n} {split} {tiles} differs from the lone run"
    for p in plans:
        p.close()
