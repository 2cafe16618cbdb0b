"""Benchmark of the QFT->FFT hot path on one MI355X.

Workload: exact QFT (DFT, forward sign, 1/sqrt(N) norm, natural output
order) of n = 28 qubits (N = 2^28 amplitudes) in complex64, input re/im
i.i.d. N(0,1) generated on the device (Philox, seed 1003) so it is resident
in HBM before the timed region.  A step is one complete transform (every
HBM pass of the fused schedule, including the final qubit-reversal
addressing and the output scale).

Prints one JSON line with the throughput as 5 N log2 N / t GFLOP/s
equivalent, the HBM roofline of the dominant kernel (measured with HIP
events around each pass during the timed region), and the FP64 oracle timed
on the host cores on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_and_accuracy(torch, Q, n, dtype, cutoff):
    """The FP64 oracle timed on the host cores on the headline workload, and
    the accuracy of the timed plan against it.

    The input is the seed-1003 N(0,1) workload drawn on the host (numpy), so
    that nothing the oracle sees comes from the device.  The GPU runs the same
    plan and kernels as the timed steps on it; the whole output is compared
    with the oracle's whole-vector per-target form (oracle.qft_state_c, the
    plain C form on every host core), and 2^20 seeded bins with the FP64
    exact DFT through the library FFT (workers = every host core), which is
    also timed as the multi-core host FFT context."""
    import numpy as np

    import oracle as O
    from paper_2606_18981_amd import inputs as I

    N = 1 << n
    k = None if cutoff < 0 else cutoff
    x = I.gaussian(n, 1003)
    npdt = np.complex64 if dtype == "c64" else np.complex128
    plan = Q.Plan(n, cutoff, "unitary", dtype, "natural")
    t = torch.from_numpy(x.astype(npdt)).cuda()
    plan.execute(t)
    torch.cuda.synchronize()
    y = t.cpu().numpy()
    del t
    plan.close()
    torch.cuda.empty_cache()

    t0 = time.perf_counter()
    ref = O.qft_state_c(x, k)
    dt_oracle = time.perf_counter() - t0
    whole = O.error_norms(y, ref)
    del ref
    nproc = os.cpu_count()
    t0 = time.perf_counter()
    exact = O.dft_library(x, workers=nproc)
    dt_fft = time.perf_counter() - t0
    bins = np.random.default_rng(1003).choice(N, min(N, 1 << 20), replace=False)
    yb = y[bins].astype(np.complex128)
    eb = exact[bins]
    del exact
    threads = O.c_oracle_threads()
    flops = 5.0 * N * n
    baseline = {
        "value": flops / dt_oracle / 1e9,
        "unit": "GFLOP/s-equiv (5N log2 N / t)",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one n={n} {'exact' if k is None else f'k={k}'} transform of the seed-1003 "
                  f"N(0,1) input: the oracle's whole-vector per-target form in FP64 "
                  f"(plain C, {threads} OpenMP threads), {dt_oracle:.2f} s",
        "seconds": dt_oracle,
        "nproc": nproc,
        "cpu_model": _cpu_model(),
        "host_fft_context": {
            "what": f"FP64 library FFT (scipy.fft, workers={nproc}) of the same input, "
                    "the exact DFT only",
            "seconds": dt_fft,
            "gflops_equiv": flops / dt_fft / 1e9,
        },
    }
    accuracy = {
        "input": f"seed-1003 N(0,1) re/im, n={n}, drawn on the host; the timed plan "
                 f"({dtype}) run once on it",
        "vs_oracle_whole_vector": {"rel_l2": whole["rel_l2"], "max_err": whole["max_err"],
                                   "elements": N},
        "vs_exact_dft_2^20_bins": {"rel_l2": O.rel_l2(yb, eb), "max_err": O.max_err(yb, eb),
                                   "bins": int(bins.size)},
        "max_err_definition": "max |y - ref| over the RMS amplitude of ref",
    }
    if k is not None:
        accuracy["expected_aqft_rel_l2_vs_exact"] = O.aqft_expected_relerr_gaussian(n, k)
    return baseline, accuracy


def pass_kernel_name(info, p, dtype):
    """Name of the kernel instance that runs pass p of a plan, as the kernel
    trace prints it (without the argument list)."""
    real = "float" if dtype == "c64" else "double"
    sh = info.pass_kernel[p]
    st = "true" if info.pass_streaming[p] else "false"
    r = info.config.radix_log2
    threads = 1 << (info.pass_bits[p] + info.pass_spec[p] - r)
    # the lean (four-wave) form: 512-thread complex64, 256-thread complex128
    wide = threads == (512 if dtype == "c64" else 256)
    if 1 <= sh <= 10:
        nst, ext = (sh - 1) % 5 + 1, "true" if sh > 5 else "false"
        return (f"k_fused_pass2w<{real}, 5, {nst}, {ext}, {st}>" if wide
                else f"k_fused_pass2<{real}, 5, {nst}, {ext}, {st}>")
    if 11 <= sh <= 16:
        s, ext = (sh - 11) % 3 + 1, "true" if sh >= 14 else "false"
        return (f"k_fused_pass3w<{real}, {s}, {ext}, {st}>" if wide
                else f"k_fused_pass3<{real}, {s}, {ext}, {st}>")
    if sh >= 17:
        return f"k_fused_pass2x<{real}, {sh - 16}, {st}>"
    return f"k_fused_pass<{real}, {r}>"


def profile_name(n, dtype, cutoff):
    tag = "exact" if cutoff < 0 else f"k{cutoff}"
    return f"fused_pass_n{n}_{dtype}_{tag}.md"


def time_plan(torch, Q, plan, x, steps, warmup):
    """Mean ms per execute (HIP events on the current stream)."""
    for _ in range(warmup):
        plan.execute(x)
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(steps):
        plan.execute(x)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def bench_aqft(torch, Q, n, dtype, cutoffs, steps):
    """Runtime of the n-qubit transform for each AQFT cutoff (and exact)."""
    N = 1 << n
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    x = torch.empty(N, dtype=tdt, device="cuda")
    Q.fill_random(x, "gaussian", seed=1003)
    rows = []
    for k in cutoffs:
        plan = Q.Plan(n, k, "unitary", dtype, "natural")
        ms = time_plan(torch, Q, plan, x, steps, 2)
        rows.append({"cutoff": k, "ms": ms, "gflops_equiv": 5.0 * N * n / (ms * 1e-3) / 1e9,
                     "hbm_gbs": plan.info.hbm_bytes / (ms * 1e-3) / 1e9,
                     "gates_cr": plan.info.gates_cr})
        plan.close()
    del x
    torch.cuda.empty_cache()
    return rows


def bench_budget(torch, Q, n, budgets, steps):
    """Cutoff picked by accuracy budget (closed-form expected error), then the
    measured error against the exact transform of the same input, taken on
    the device by the transform's own last pass (Plan.execute with ref:
    qft_execute_compare), and the runtime of the picked AQFT: alone, with
    the metrics taken in its last pass, and followed by the separate
    comparison pass (qft_compare) instead."""
    N = 1 << n
    x = torch.empty(N, dtype=torch.complex64, device="cuda")
    Q.fill_random(x, "gaussian", seed=1003)
    exact = x.clone()
    plan = Q.Plan(n, -1, "unitary", "c64", "natural")
    plan.execute(exact)
    plan.close()
    mo = torch.empty(len(Q.METRIC_NAMES), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(1, int(Q.lib.qft_compare_workspace_bytes(n)) // 8), dtype=torch.float64,
                     device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / steps

    rows = []
    for budget in budgets:
        k = Q.select_cutoff(n, budget)
        plan = Q.Plan(n, k, "unitary", "c64", "natural")
        y = x.clone()
        plan.execute(y, ref=exact, metrics_out=mo)
        m = Q.metrics_dict(mo)
        sep = Q.compare(y, exact, workspace=ws)  # the same output, the separate pass
        ms = time_plan(torch, Q, plan, y, steps, 2)  # (transforms y in place)
        ms_fused = timed(lambda: plan.execute(y, ref=exact, metrics_out=mo))
        ms_sep = timed(lambda: (plan.execute(y),
                                Q.compare(y, exact, workspace=ws, out=mo, as_dict=False)))
        del y
        rows.append({"budget": budget, "cutoff": k, "predicted_rel_l2": Q.expected_error(n, k),
                     "measured_rel_l2": m["rel_l2"], "fidelity": m["fidelity"],
                     "leakage": m["leakage"], "max_err": m["max_err"],
                     "separate_pass_rel_l2": sep["rel_l2"],
                     "ms": ms, "ms_with_metrics_in_last_pass": ms_fused,
                     "ms_then_separate_compare": ms_sep, "gates_cr": plan.info.gates_cr})
        plan.close()
    del x, exact, ws
    torch.cuda.empty_cache()
    return rows


def bench_circuit(torch, Q, n=24, steps=5):
    """The QFT written as general gates (H, controlled phases, swaps) and run
    through the general fused-circuit path, against the QFT plan."""
    import numpy as np
    N = 1 << n
    x = torch.empty(N, dtype=torch.complex64, device="cuda")
    Q.fill_random(x, "gaussian", seed=1003)
    c = Q.Circuit(n, "c64")
    h = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    for t in range(n - 1, -1, -1):
        c.add_1q(t, h)
        for d in range(1, t + 1):
            c.add_controlled(t - d, t, np.diag([1.0, np.exp(-2j * np.pi / 2.0 ** (d + 1))]))
    for a in range(n // 2):
        c.add_swap(a, n - 1 - a)
    c.compile()
    info = c.info()
    for _ in range(2):
        c.execute(x)
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(steps):
        c.execute(x)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / steps
    c.close()
    plan = Q.Plan(n, -1, "unitary", "c64", "natural")
    ms_plan = time_plan(torch, Q, plan, x, 10, 2)
    plan.close()
    del x
    torch.cuda.empty_cache()
    return {"n": n, "gates": info["gates"], "passes": info["passes"], "ms": ms,
            "gbs": info["passes"] * 2 * N * 8 / (ms * 1e-3) / 1e9,
            "qft_plan_ms": ms_plan, "qft_plan_passes": 3}


def bench_gate_schedule(torch, Q, n=24, steps=3):
    """The same transform run gate by gate (one HBM sweep per H, controlled
    phase and swap, the unfused form) against the fused plan."""
    N = 1 << n
    x = torch.empty(N, dtype=torch.complex64, device="cuda")
    Q.fill_random(x, "gaussian", seed=1003)
    rows = {}
    for schedule in ("gates", "fused"):
        plan = Q.Plan(n, -1, "unitary", "c64", "natural", schedule)
        ms = time_plan(torch, Q, plan, x, steps, 1)
        info = plan.info
        gates = info.gates_h + info.gates_cr + info.gates_swap
        rows[schedule] = {"ms": ms, "passes": info.num_passes if schedule == "fused" else gates,
                          "hbm_bytes": info.hbm_bytes, "bytes_per_gate": info.hbm_bytes / gates,
                          "hbm_gbs": info.hbm_bytes / (ms * 1e-3) / 1e9}
        plan.close()
    del x
    torch.cuda.empty_cache()
    rows["n"] = n
    rows["gate_count"] = gates
    rows["speedup_fused"] = rows["gates"]["ms"] / rows["fused"]["ms"]
    return rows


def bench_configs(torch, Q):
    """The small configurations: n = 10 complex128 (gate by gate and fused,
    launch-bound, microseconds), n = 12, 14 and 22 complex64 and n = 24 in
    both element types."""
    rows = []
    # n = 12, 14 and 22 complex64 are the sizes the paper times (FP32)
    for n, dtype, schedule, steps in ((10, "c128", "gates", 200), (10, "c128", "fused", 200),
                                      (12, "c64", "fused", 200), (14, "c64", "fused", 200),
                                      (22, "c64", "fused", 50),
                                      (24, "c64", "fused", 20), (24, "c128", "fused", 20)):
        N = 1 << n
        x = torch.empty(N, dtype=torch.complex64 if dtype == "c64" else torch.complex128,
                        device="cuda")
        Q.fill_random(x, "uniform" if n <= 14 else "gaussian", seed=1001 if n <= 14 else 1002)
        plan = Q.Plan(n, -1, "unitary", dtype, "natural", schedule)
        ms = time_plan(torch, Q, plan, x, steps, 5)
        info = plan.info
        # one launch per gate sweep (the unitary norm needs no scaling sweep)
        launches = info.num_passes if schedule == "fused" else (
            info.gates_h + info.gates_cr + info.gates_swap)
        rows.append({"n": n, "dtype": dtype, "schedule": schedule, "us": ms * 1e3,
                     "launches": launches, "gflops_equiv": 5.0 * N * n / (ms * 1e-3) / 1e9,
                     "hbm_gbs": info.hbm_bytes / (ms * 1e-3) / 1e9})
        plan.close()
        del x
    torch.cuda.empty_cache()
    return rows


def bench_sizes(torch, Q, sizes=range(24, 31), reps=5):
    """Exact transforms across sizes in both element types: the sum of the
    per-pass HIP-event times (mean over `reps` executes, best of three), as
    a fraction of 8 TB/s both for the plan's own passes and for the
    three-pass floor 2*3*N*S (a plan with an extra pass moves more)."""
    rows = []
    for dtype in ("c64", "c128"):
        for n in sizes:
            N = 1 << n
            x = torch.empty(N, dtype=torch.complex64 if dtype == "c64" else torch.complex128,
                            device="cuda")
            Q.fill_random(x, "gaussian", seed=1002)
            plan = Q.Plan(n, -1, "unitary", dtype, "natural")
            info = plan.info
            for _ in range(2):
                plan.execute(x)
            best = None
            for _ in range(3):
                torch.cuda.synchronize()
                plan.set_timing(True)
                for _ in range(reps):
                    plan.execute(x)
                torch.cuda.synchronize()
                ms, _ = plan.pass_times()
                plan.set_timing(False)
                if best is None or sum(ms) < sum(best):
                    best = ms
            t = sum(best) * 1e-3
            S = 8 if dtype == "c64" else 16
            rows.append({"n": n, "dtype": dtype, "ms": sum(best),
                         "pass_bits": list(info.pass_bits)[:info.num_passes],
                         "pass_ms": best,
                         "frac_plan": info.hbm_bytes / t / 1e9 / HBM_PEAK_GBS,
                         "frac_three_pass_floor": 6 * N * S / t / 1e9 / HBM_PEAK_GBS,
                         "dominant_pass_frac": 2 * N * S / (max(best) * 1e-3) / 1e9 / HBM_PEAK_GBS})
            plan.close()
            del x
            torch.cuda.empty_cache()
    return rows


def bench_batch(torch, Q, reps=10):
    """512 uneven transforms: the batched launches in one HIP graph, the same
    launches enqueued directly, and one plan execute per transform, with the
    default configuration; then the configuration the batch autotuner picks
    for the whole batch (qft_tune_batch), in the graph."""
    from paper_2606_18981_amd import inputs as I
    ns, cuts = I.batch_sizes(1004, count=512, lo=8, hi=20, aqft_frac=0.25, aqft_k=8)
    xs = []
    for i, n in enumerate(ns.tolist()):
        t = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
        Q.fill_random(t, "uniform", seed=1004 + i)
        xs.append(t)
    elems = sum(1 << n for n in ns.tolist())
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)

    def make_plans(config):
        cache, plans = {}, []
        for n, k in zip(ns.tolist(), cuts.tolist()):
            if (n, k) not in cache:
                cache[(n, k)] = Q.Plan(n, k, "unitary", "c64", "natural", config=config)
            plans.append(cache[(n, k)])
        return cache, plans

    def timed(run):
        run()
        torch.cuda.synchronize()
        s.record()
        for _ in range(reps):
            run()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps

    cache, plans = make_plans(None)
    batch = Q.Batch(plans, xs)  # arguments checked and marshalled once
    total_bytes = sum(p.info.hbm_bytes for p in plans)
    res = {"transforms": 512, "total_amplitudes": int(elems),
           "algorithmic_hbm_bytes": int(total_bytes)}
    for mode in ("graph", "eager", "per_launch"):
        def run():
            if mode == "per_launch":
                for p, t in zip(plans, xs):
                    p.execute(t)
            else:
                batch.execute(graph=(mode == "graph"))
        ms = timed(run)
        res[mode] = {"ms": ms, "transforms_per_s": 512 / (ms * 1e-3),
                     "hbm_gbs": total_bytes / (ms * 1e-3) / 1e9}
    res["speedup_graph_vs_per_launch"] = res["per_launch"]["ms"] / res["graph"]["ms"]
    for p in cache.values():
        p.close()
    # the batch autotuner: one configuration for the whole batch
    t0 = time.perf_counter()
    best, tune_ms = Q.tune_batch(ns.tolist(), cuts.tolist(), xs, reps=3)
    tune_s = time.perf_counter() - t0
    cache, plans = make_plans(best)
    tuned_bytes = sum(p.info.hbm_bytes for p in plans)
    batch = Q.Batch(plans, xs)
    ms = timed(lambda: batch.execute(graph=True))
    res["tuned"] = {"config": best, "tuner_seconds": tune_s, "tuner_ms": tune_ms,
                    "graph": {"ms": ms, "transforms_per_s": 512 / (ms * 1e-3),
                              "algorithmic_hbm_bytes": int(tuned_bytes),
                              "hbm_gbs": tuned_bytes / (ms * 1e-3) / 1e9}}
    res["speedup_tuned_vs_default_graph"] = res["graph"]["ms"] / ms
    for p in cache.values():
        p.close()
    del xs
    torch.cuda.empty_cache()
    return res


def bench_serve(torch, Q, seconds, rate=2000.0, sweep_rates=(4000.0, 6000.0, 8000.0, 12000.0),
                sweep_seconds=4.0):
    """Poisson request streams: continuous batching (64 slots over 4 streams)
    against one transform at a time (1 slot, 1 stream), on the config's trace
    (2000 requests/s for `seconds`) and on shorter traces at higher rates,
    to find where one at a time saturates."""
    from paper_2606_18981_amd import inputs as I
    from paper_2606_18981_amd import serve as S
    budget = 200 << 30

    def run_modes(rate, seconds):
        trace = I.served_trace(1005, rate=rate, duration=seconds, n_lo=10, n_hi=26)
        reqs = S.requests_from_trace(trace)
        out = {"requests": len(reqs), "rate_per_s": rate, "seconds": seconds}
        for name, slots, streams in (("continuous", 64, 4), ("one_at_a_time", 1, 1)):
            srv = S.Server(budget, slots, streams)
            srv.prepare(reqs)
            res, st = srv.run(reqs)
            summ = S.latency_summary(res)
            summ.update({"completed": st["completed"], "failed": st["failed"],
                         "peak_inflight": st["peak_inflight"],
                         "peak_reserved_gb": st["peak_reserved_bytes"] / 1e9,
                         "plan_tables_gb": st["plan_bytes"] / 1e9,
                         "wall_s": st["wall_seconds"],
                         "requests_per_s": st["completed"] / st["wall_seconds"],
                         "hbm_gbs": st["hbm_bytes"] / st["wall_seconds"] / 1e9})
            out[name] = summ
            srv.close()
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            print(f"[bench] serve {rate:.0f}/s {seconds:g} s {name}: p50 "
                  f"{summ.get('p50_ms', 0):.3f} ms p99 {summ.get('p99_ms', 0):.3f} ms",
                  file=sys.stderr, flush=True)
        return out

    out = {"budget_bytes": budget, "trace": run_modes(rate, seconds)}
    out["rate_sweep"] = [run_modes(r, sweep_seconds) for r in sweep_rates]
    return out


EXTRA_LEGS = ("configs", "sizes", "aqft", "budget", "c128", "gates", "circuit", "batch", "serve")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--cutoff", type=int, default=-1)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline measurement")
    ap.add_argument("--extras", default="all",
                    help="comma-separated legs after the headline: " + ",".join(EXTRA_LEGS))
    ap.add_argument("--copy-ref", action="store_true",
                    help="also time a plain device copy of the state (read + write of "
                         "N*S bytes each) as the reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    legs = set(EXTRA_LEGS) if args.extras == "all" else set(args.extras.split(","))
    unknown = legs - set(EXTRA_LEGS)
    if unknown:
        print(f"unknown --extras legs {sorted(unknown)}; known: {', '.join(EXTRA_LEGS)}",
              file=sys.stderr)
        sys.exit(2)
    if args.no_extras:
        legs = set()

    import torch

    from paper_2606_18981_amd import qft as Q

    n = args.n
    N = 1 << n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    plan = Q.Plan(n, args.cutoff, "unitary", args.dtype, "natural")
    info = plan.info
    x = torch.empty(N, dtype=tdt, device=dev)
    stream = torch.cuda.current_stream()
    Q.fill_random(x, "gaussian", seed=1003, stream_id=0)
    torch.cuda.synchronize()
    print(f"[bench] n={n} dtype={args.dtype} cutoff={args.cutoff} passes={info.num_passes} "
          f"pass_bits={list(info.pass_bits)[:info.num_passes]} warmup={args.warmup} "
          f"steps={args.steps}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.execute(x)
    torch.cuda.synchronize()

    plan.set_timing(True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        plan.execute(x)
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    pass_ms, execs = plan.pass_times()
    plan.set_timing(False)
    assert execs == args.steps

    ms_per_step = total_ms / args.steps
    flops = 5.0 * N * n
    gflops = flops / (ms_per_step * 1e-3) / 1e9
    state_bytes = info.state_bytes
    per_launch_bytes = 2 * state_bytes  # one read and one write of the state
    names = [pass_kernel_name(info, p, args.dtype) for p in range(info.num_passes)]
    # every pass is one launch of a pass kernel instance; the dominant kernel
    # is the slowest pass (HIP events on the launch stream, timed region)
    per_pass = [{"pass": p, "kernel": names[p], "qubits": info.pass_bits[p],
                 "ms": pass_ms[p],
                 "gbs": per_launch_bytes / (pass_ms[p] * 1e-3) / 1e9,
                 "frac": per_launch_bytes / (pass_ms[p] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                for p in range(info.num_passes)]
    dom = max(range(info.num_passes), key=lambda p: pass_ms[p])
    achieved = per_pass[dom]["gbs"]
    mean_pass_ms = sum(pass_ms) / len(pass_ms)
    hbm_gbs = info.hbm_bytes / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": "5N*log2N/t GFLOP/s-equiv + HBM GB/s at n=28; p50/p99 latency under load",
        "value": gflops,
        "unit": "GFLOP/s-equiv",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if args.dtype == "c64" else "c128",
        "data": "synthetic: re/im i.i.d. N(0,1) from the device Philox generator, seed 1003",
        "config": {
            "workload": f"exact QFT->DFT, n={n} ({N} amplitudes), complex"
                        f"{64 if args.dtype == 'c64' else 128}, unitary norm, natural order, "
                        f"cutoff={args.cutoff}",
            "n": n, "cutoff": args.cutoff, "passes": info.num_passes,
            "pass_bits": list(info.pass_bits)[:info.num_passes],
            "kernel_config": Q._cfg_dict(info.config),
        },
        "hbm_gbs": hbm_gbs,
        "hbm_frac_whole_step": hbm_gbs / HBM_PEAK_GBS,
        "pass_ms": pass_ms,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": names[dom],
            "dominant": f"pass {dom} ({info.pass_bits[dom]} qubits), the slowest of the plan's "
                        f"{info.num_passes} pass launches",
            "algorithmic_bytes_per_launch": per_launch_bytes,
            "per_pass": per_pass,
            "mean_pass_frac": per_launch_bytes / (mean_pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
    }
    # HBM traffic of the dominant kernel from the committed rocprofv3 counter
    # summary of this same workload and kernel sources (FETCH_SIZE and
    # WRITE_SIZE, each scaled by what it reads for a plain device copy of
    # known size); null otherwise
    from paper_2606_18981_amd import profile_summary as PS
    prof = os.path.join(ROOT, "profiles", profile_name(n, args.dtype, args.cutoff))
    tr = PS.load_traffic(prof, out["config"], names[dom])
    out["roofline"]["traffic"] = tr
    out["roofline"]["traffic_source"] = os.path.relpath(prof, ROOT)
    # HBM bytes per gate of the circuit (H, controlled phases, swaps): the
    # fused plan's passes shared over its gates, from the algorithmic bytes
    # and from the counters; a gate-by-gate sweep moves 2*N*S per gate
    gates = info.gates_h + info.gates_cr + info.gates_swap
    plan_traffic = PS.load_plan_traffic(prof, out["config"])
    out["bytes_per_gate"] = {
        "gates": {"h": info.gates_h, "controlled_phase": info.gates_cr,
                  "swap": info.gates_swap},
        "algorithmic": info.hbm_bytes / gates,
        "counters": plan_traffic / gates if plan_traffic else None,
        "gate_by_gate_sweep": per_launch_bytes,
    }
    if args.copy_ref:
        y = torch.empty_like(x)
        ms_copy = None
        for _ in range(3):
            y.copy_(x)
        cs = torch.cuda.Event(enable_timing=True)
        ce = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        cs.record()
        for _ in range(10):
            y.copy_(x)
        ce.record()
        torch.cuda.synchronize()
        ms_copy = cs.elapsed_time(ce) / 10
        out["copy_ref"] = {"bytes_read": state_bytes, "bytes_written": state_bytes,
                           "ms": ms_copy, "gbs": 2 * state_bytes / (ms_copy * 1e-3) / 1e9}
        del y
    plan.close()
    del x
    torch.cuda.empty_cache()
    if "configs" in legs:
        print("[bench] n = 10 and n = 24", file=sys.stderr, flush=True)
        out["small_configs"] = bench_configs(torch, Q)
    if "sizes" in legs:
        print("[bench] sizes n = 24..30", file=sys.stderr, flush=True)
        out["sizes"] = bench_sizes(torch, Q)
    if "aqft" in legs:
        print("[bench] aqft sweep", file=sys.stderr, flush=True)
        out["aqft_n28_c64"] = bench_aqft(torch, Q, 28, "c64", [-1, 6, 10, 14, 18], 10)
        out["aqft_n30_c64"] = bench_aqft(torch, Q, 30, "c64", [-1, 6, 10, 14, 18], 10)
    if "budget" in legs:
        print("[bench] cutoff by accuracy budget", file=sys.stderr, flush=True)
        out["aqft_budget_n28_c64"] = bench_budget(torch, Q, 28, [1e-2, 1e-3, 1e-4], 10)
    if "c128" in legs:
        print("[bench] complex128", file=sys.stderr, flush=True)
        out["exact_n28_c128"] = bench_aqft(torch, Q, 28, "c128", [-1], 10)[0]
    if "gates" in legs:
        print("[bench] gate-by-gate schedule", file=sys.stderr, flush=True)
        out["gate_schedule_n24_c64"] = bench_gate_schedule(torch, Q)
    if "circuit" in legs:
        print("[bench] general circuit", file=sys.stderr, flush=True)
        out["general_circuit_qft_n24_c64"] = bench_circuit(torch, Q)
    if "batch" in legs:
        print("[bench] batch", file=sys.stderr, flush=True)
        out["batch_512"] = bench_batch(torch, Q)
    if "serve" in legs:
        print("[bench] serve", file=sys.stderr, flush=True)
        out["serve"] = bench_serve(torch, Q, args.serve_seconds)
        out["p50_ms"] = out["serve"]["trace"]["continuous"].get("p50_ms")
        out["p99_ms"] = out["serve"]["trace"]["continuous"].get("p99_ms")
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline and accuracy of the timed plan", file=sys.stderr, flush=True)
        out["cpu_baseline"], out["accuracy"] = cpu_baseline_and_accuracy(
            torch, Q, n, args.dtype, args.cutoff)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
