"""qft_execute_norm_static (the entry point that allocates nothing: its
partial sums live in a static device array) against qft_execute_norm, through
the C ABI: the transformed state bitwise equal and the same norm, on two
calls in a row, the second with a smaller input; the refusal of a plan that
needs more partial sums than the array holds."""

import ctypes

import numpy as np
import pytest

from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_norm_static_matches_allocating_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_18981_amd import qft as Q
    lib = Q.lib
    # (n, dtype, schedule): a fused three-pass plan, then a smaller one-pass
    # plan, then a gate-schedule plan (its own norm sweep)
    for n, dtype, schedule in ((22, "c64", "fused"), (9, "c128", "fused"), (12, "c64", "gates")):
        print(f"[gpu] norm_static n={n} {dtype} {schedule}", flush=True)
        npdt = np.complex64 if dtype == "c64" else np.complex128
        x = (I.gaussian(n, 9100 + n) * 2.5).astype(npdt)
        plan = Q.Plan(n, -1, "unitary", dtype, "natural", schedule)
        a = torch.from_numpy(x).cuda()
        b = a.clone()
        na = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        nb = torch.full((1,), -2.0, dtype=torch.float64, device="cuda")
        rc = lib.qft_execute_norm(plan.handle, ctypes.c_void_p(a.data_ptr()), None,
                                  ctypes.c_void_p(na.data_ptr()), None)
        assert rc == 0, Q.last_error()
        rc = lib.qft_execute_norm_static(plan.handle, ctypes.c_void_p(b.data_ptr()), None,
                                         ctypes.c_void_p(nb.data_ptr()), None)
        assert rc == 0, Q.last_error()
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert float(na.cpu()[0]) == float(nb.cpu()[0])
        ref = float(np.linalg.norm(x.astype(np.complex128)))
        assert abs(float(nb.cpu()[0]) - ref) <= (1e-13 if dtype == "c128" else 1e-6) * ref
        # NULL norm pointer refused, nothing launched
        rc = lib.qft_execute_norm_static(plan.handle, ctypes.c_void_p(b.data_ptr()), None, None,
                                         None)
        assert rc == Q.QFT_ERR_POINTER
        plan.close()


def test_norm_static_refuses_plans_beyond_the_array():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_18981_amd import qft as Q
    # 2^23 elements in tiles of 2^6 with two threads each (radix 5): one
    # partial per thread, 2^18 tiles x 2 = 2^18 partials fit; 2^26 elements
    # need 2^21 partials, beyond the 2^20 the array holds
    cfg = dict(tile_log2=6, radix_log2=5, spec_log2=1, rev_spec_log2=1)
    plan = Q.Plan(26, -1, "unitary", "c64", "bitrev", "fused", cfg, workspace=False)
    t = torch.empty(1 << 26, dtype=torch.complex64, device="cuda")
    nrm = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = Q.lib.qft_execute_norm_static(plan.handle, ctypes.c_void_p(t.data_ptr()), None,
                                       ctypes.c_void_p(nrm.data_ptr()), None)
    assert rc == Q.QFT_ERR_UNSUPPORTED
    assert "static scratch" in Q.last_error()
    plan.close()
