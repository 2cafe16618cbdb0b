"""On-device accuracy metrics (qft_compare) against the oracle's metrics on
the same arrays, and cutoff selection checked by measurement."""

import ctypes

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

NPDT = {"c64": np.complex64, "c128": np.complex128}


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_18981_amd import qft as Q
    return torch, Q


def transform(torch, Q, x, n, k, dtype):
    plan = Q.Plan(n, k, "unitary", dtype, "natural")
    t = torch.from_numpy(x.astype(NPDT[dtype])).cuda()
    plan.execute(t)
    plan.close()
    return t


def oracle_metrics(y, ref):
    y = y.astype(np.complex128)
    ref = ref.astype(np.complex128)
    return {"rel_l2": O.rel_l2(y, ref), "max_err": O.max_err(y, ref),
            "fidelity": O.fidelity(y, ref), "leakage": O.top_bin_leakage(y, ref),
            "norm_y": float(np.linalg.norm(y)), "norm_ref": float(np.linalg.norm(ref)),
            "argmax": int(np.argmax(np.abs(ref)))}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,k,which", [(16, 5, "gaussian"), (12, 3, "tone"), (20, 8, "tones"),
                                       (1, 0, "gaussian"), (6, 2, "gaussian")])
def test_compare_matches_oracle(env, dtype, n, k, which):
    torch, Q = env
    print(f"[gpu] compare n={n} k={k} {which} {dtype}", flush=True)
    if which == "gaussian":
        x = I.gaussian(n, 8000 + n)
    elif which == "tone":
        x = I.tone(n, 37 % (1 << n))
    else:
        x = I.multi_tone(n, 8100, 4, 0.01)[0]
    y = transform(torch, Q, x, n, k, dtype)
    ref = transform(torch, Q, x, n, -1, dtype)
    torch.cuda.synchronize()
    got = Q.compare(y, ref)
    want = oracle_metrics(y.cpu().numpy(), ref.cpu().numpy())
    for key in ("rel_l2", "max_err", "fidelity", "leakage", "norm_y", "norm_ref"):
        assert got[key] == pytest.approx(want[key], rel=1e-9, abs=1e-12), key
    assert got["argmax"] == want["argmax"]
    # deterministic: a second call gives the same bits
    again = Q.compare(y, ref)
    assert again == got


def test_compare_errors(env):
    torch, Q = env
    a = torch.zeros(1 << 10, dtype=torch.complex64, device="cuda")
    ws = torch.empty(64, dtype=torch.float64, device="cuda")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    rc = Q.lib.qft_compare(ctypes.c_void_p(a.data_ptr()), None, 10, Q.QFT_C64,
                           ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(out.data_ptr()), None)
    assert rc == Q.QFT_ERR_POINTER
    rc = Q.lib.qft_compare(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(a.data_ptr()), 40,
                           Q.QFT_C64, ctypes.c_void_p(ws.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), None)
    assert rc == Q.QFT_ERR_INVALID


def test_selected_cutoff_meets_budget(env):
    # pick k by the closed form, then measure the AQFT against the exact
    # transform on the device: the measured error sits at the prediction
    torch, Q = env
    n = 22
    x = I.gaussian(n, 8200)
    ref = transform(torch, Q, x, n, -1, "c128")
    for budget in (3e-2, 1e-3, 1e-5):
        k = Q.select_cutoff(n, budget)
        print(f"[gpu] budget {budget} -> k={k}", flush=True)
        y = transform(torch, Q, x, n, k, "c128")
        m = Q.compare(y, ref)
        pred = Q.expected_error(n, k)
        assert m["rel_l2"] <= budget * 1.05
        assert m["rel_l2"] == pytest.approx(pred, rel=0.05)
