"""GPU tests of the batched launch (uneven sizes, level-by-level group launches in one graph,
one-pass transforms on a stream of their own).

Each transform in a batch must give exactly the result of running it alone
(same kernels, same arithmetic) and agree with the FP64 oracle.  Graph
replays are interleaved with eager work and each replay is checked.
"""

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I

pytestmark = pytest.mark.gpu

def within(y, ref, tol):
    """Relative L2 and max error over the RMS amplitude both <= tol."""
    e = O.error_norms(y, ref)
    return e["rel_l2"] <= tol and e["max_err"] <= tol


TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2606_18981_amd import qft as Q
    assert torch.cuda.is_available()
    return torch, Q


def make_batch(torch, Q, ns, cuts, dtype, seed, order="natural"):
    plans, xs, hosts = [], [], []
    cache = {}
    for i, (n, k) in enumerate(zip(ns.tolist(), cuts.tolist())):
        key = (n, k)
        if key not in cache:
            cache[key] = Q.Plan(n, k, "unitary", dtype, order)
        plans.append(cache[key])
        x = I.uniform_pm1(n, seed + i)
        hosts.append(x)
        xs.append(torch.from_numpy(x.astype(NPDT[dtype])).cuda())
    return plans, xs, hosts, cache


def alone(torch, Q, plans, hosts, dtype):
    out = []
    for p, x in zip(plans, hosts):
        t = torch.from_numpy(x.astype(NPDT[dtype])).cuda()
        p.execute(t)
        out.append(t)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_alone_and_oracle(env, dtype, graph):
    torch, Q = env
    ns, cuts = I.batch_sizes(1004, count=64, lo=8, hi=16, aqft_frac=0.25, aqft_k=8)
    print(f"[gpu] batch 64 dtype={dtype} graph={graph} n={ns.tolist()}", flush=True)
    plans, xs, hosts, cache = make_batch(torch, Q, ns, cuts, dtype, 500)
    ref_alone = alone(torch, Q, plans, hosts, dtype)
    Q.execute_batch(plans, xs, graph=graph)
    torch.cuda.synchronize()
    for i, (t, x, n, k) in enumerate(zip(xs, hosts, ns.tolist(), cuts.tolist())):
        y = t.cpu().numpy()
        assert np.array_equal(y, ref_alone[i]), f"item {i} (n={n}, k={k}) differs from alone"
        if i % 4 == 0:
            ref = O.qft_fused_targets(x, None if k < 0 else k)
            assert within(y, ref, TOL[dtype])
    for p in cache.values():
        p.close()


def test_graph_replays_with_eager_work_between(env):
    torch, Q = env
    dtype = "c64"
    ns = np.array([8, 12, 14, 17, 20, 9, 15, 18])
    cuts = np.array([-1, 8, -1, -1, 8, -1, 3, -1])
    plans, xs, hosts, cache = make_batch(torch, Q, ns, cuts, dtype, 900)
    ref_alone = alone(torch, Q, plans, hosts, dtype)
    for rep in range(4):
        print(f"[gpu] graph replay {rep}", flush=True)
        # eager work between replays: refill the inputs
        for t, x in zip(xs, hosts):
            t.copy_(torch.from_numpy(x.astype(np.complex64)))
        junk = torch.randn(1 << 20, device="cuda").sum()
        Q.execute_batch(plans, xs, graph=True)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for i, t in enumerate(xs):
            assert np.array_equal(t.cpu().numpy(), ref_alone[i]), f"replay {rep} item {i}"
    for p in cache.values():
        p.close()


def test_full_uneven_batch_512(env):
    """The batched workload: 512 transforms, n log-uniform in [8, 20],
    25% AQFT k = 8, complex64, uniform[-1, 1] inputs."""
    torch, Q = env
    ns, cuts = I.batch_sizes(1004, count=512, lo=8, hi=20, aqft_frac=0.25, aqft_k=8)
    print(f"[gpu] batch 512 total elements {int(sum(1 << int(n) for n in ns))}", flush=True)
    plans, xs, hosts, cache = make_batch(torch, Q, ns, cuts, "c64", 4000)
    ref_alone = alone(torch, Q, plans, hosts, "c64")
    Q.execute_batch(plans, xs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    sample = set(rng.choice(512, 24, replace=False).tolist())
    for i, t in enumerate(xs):
        y = t.cpu().numpy()
        assert np.array_equal(y, ref_alone[i])
        if i in sample:
            k = int(cuts[i])
            ref = O.qft_fused_targets(hosts[i], None if k < 0 else k)
            assert within(y, ref, 1e-5)
    for p in cache.values():
        p.close()


def test_batch_with_inverse_plans(env):
    torch, Q = env
    ns = [10, 14, 17, 12, 19, 9]
    ks = [-1, -1, 6, 3, -1, -1]
    inv = [True, False, True, False, True, True]
    plans, xs, hosts = [], [], []
    for i, (n, k, v) in enumerate(zip(ns, ks, inv)):
        plans.append(Q.Plan(n, k, "unitary", "c64", "natural", inverse=v))
        x = I.uniform_pm1(n, 7000 + i)
        hosts.append(x)
        xs.append(torch.from_numpy(x.astype(np.complex64)).cuda())
    print(f"[gpu] batch with inverse plans n={ns}", flush=True)
    Q.execute_batch(plans, xs, graph=True)
    torch.cuda.synchronize()
    for t, x, n, k, v in zip(xs, hosts, ns, ks, inv):
        ref = O.qft_fused_targets(x, None if k < 0 else k, inverse=v)
        assert within(t.cpu().numpy(), ref, 1e-5)
    for p in plans:
        p.close()


def test_cache_bound_evicts_oldest(env):
    """More than 64 distinct (plans, pointers) sets: the oldest cached sets
    are released and every call still gives the result of running alone."""
    torch, Q = env
    plan = Q.Plan(10, -1, "unitary", "c64", "natural")
    x = I.uniform_pm1(10, 4242)
    ref = alone(torch, Q, [plan], [x], "c64")[0]
    keep = []  # every tensor stays alive, so each call is a new pointer set
    for i in range(70):
        t = torch.from_numpy(x.astype(np.complex64)).cuda()
        keep.append(t)
        Q.execute_batch([plan], [t], graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), ref), f"set {i}"
    assert len({t.data_ptr() for t in keep}) == 70
    # the first (evicted) set runs again, rebuilt
    t0 = keep[0]
    t0.copy_(torch.from_numpy(x.astype(np.complex64)))
    Q.execute_batch([plan], [t0], graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(t0.cpu().numpy(), ref)
    plan.close()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_handle_replays(env, graph):
    # the reusable Batch handle (arguments marshalled once) gives the lone
    # results bit for bit on every replay, one-pass and multi-pass transforms
    # mixed (the one-pass ones run on their own stream)
    torch, Q = env
    ns, cuts = I.batch_sizes(1004, count=64, lo=8, hi=18, aqft_frac=0.25, aqft_k=8)
    plans, xs, hosts, cache = make_batch(torch, Q, ns, cuts, "c64", 8100)
    ref = alone(torch, Q, plans, hosts, "c64")
    b = Q.Batch(plans, xs)
    for rep in range(3):
        for t, x in zip(xs, hosts):
            t.copy_(torch.from_numpy(x.astype(np.complex64)))
        print(f"[gpu] batch handle graph={graph} replay {rep}", flush=True)
        b.execute(graph=graph)
        torch.cuda.synchronize()
        for i, (t, r) in enumerate(zip(xs, ref)):
            assert np.array_equal(t.cpu().numpy(), r), f"transform {i} (n={ns[i]}) replay {rep}"
    for p in cache.values():
        p.close()
