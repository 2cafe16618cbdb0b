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


def cpu_baseline(n_sample: int = 24):
    """Time the FP64 oracle (per-target fused numpy form) on one transform."""
    import numpy as np

    import oracle as O
    from paper_2606_18981_amd import inputs as I

    x = I.gaussian(n_sample, 1003)
    t0 = time.perf_counter()
    O.qft_fused_targets(x, None, "unitary", "natural")
    dt = time.perf_counter() - t0
    N = 1 << n_sample
    return {
        "value": 5.0 * N * n_sample / dt / 1e9,
        "unit": "GFLOP/s-equiv (5N log2 N / t)",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one exact n={n_sample} complex128 transform (oracle per-target fused form, "
                  f"numpy FP64, single thread), {dt:.2f} s",
        "seconds": dt,
        "nproc": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--cutoff", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

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
    # dominant kernel: every pass launches the same fused-pass kernel; the
    # roofline uses its mean launch time over the timed region
    mean_pass_ms = sum(pass_ms) / len(pass_ms)
    achieved = per_launch_bytes / (mean_pass_ms * 1e-3) / 1e9
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
            "kernel_config": {f: getattr(info.config, f) for f, _ in Q.Config._fields_},
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
            "kernel": "k_fused_pass (mean over the plan's passes)",
            "algorithmic_bytes_per_launch": per_launch_bytes,
        },
    }
    plan.close()
    del x
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
