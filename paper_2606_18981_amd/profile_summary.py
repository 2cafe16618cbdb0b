"""Summarise rocprofv3 results of a bench run as a short markdown file.

Reads the SQLite result databases that ``rocprofv3 -d DIR -o run`` writes
(one kernel-trace run and two counter runs, FETCH_SIZE and WRITE_SIZE), and
prints: the per-kernel duration statistics, the counters per dispatch, the
scale factors that make the counters read true bytes on a plain device copy
of known size, and one JSON block that ``bench.py`` reads back to report the
HBM traffic of the pass kernel.  The JSON block records a digest of the
kernel and planner sources; the traffic figure is only used while the
sources still have that digest.

Usage (from the repository root)::

    python -m paper_2606_18981_amd.profile_summary \
        --trace out/prof/trace --fetch out/prof/fetch \
        --write out/prof/write --copy-bytes 2147483648 \
        --cmd-trace "..." --cmd-fetch "..." --cmd-write "..." \
        --bench-json out/prof/trace.log > profiles/<name>.md
"""

import argparse
import collections
import glob
import hashlib
import json
import os
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))

# Sources whose change can change what the pass kernel reads and writes.
KERNEL_SOURCES = (
    "csrc/qft_kernels.hip",
    "csrc/qft_kernels.h",
    "csrc/qft_pass_tile.h",
    "csrc/qft_internal.h",
    "csrc/qft_planner.cpp",
    "csrc/qft_planner.h",
    "build.py",  # the compiler flags
)

PASS_PREFIX = "void qft::k_fused_pass"
COPY_NAME = "__amd_rocclr_copyBuffer"


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _db(path):
    if os.path.isdir(path):
        cands = sorted(glob.glob(os.path.join(path, "**", "*results.db"), recursive=True))
        if not cands:
            raise FileNotFoundError(f"no *results.db under {path}")
        path = cands[0]
    return sqlite3.connect(path)


def kernel_stats(path):
    """Per-kernel dispatch count and duration statistics (ns), from the
    per-dispatch `kernels` view, ordered by total time."""
    cur = _db(path).cursor()
    rows = cur.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                       "max(duration), max(vgpr_count), max(accum_vgpr_count), "
                       "max(scratch_size), max(lds_size) from kernels group by name "
                       "order by sum(duration) desc").fetchall()
    return [dict(name=r[0], calls=r[1], total_ns=r[2], avg_ns=r[3], min_ns=r[4], max_ns=r[5],
                 vgpr=r[6], agpr=r[7], scratch=r[8], lds=r[9]) for r in rows]


def counter_means(path, counter):
    """Mean counter value per (kernel, grid) over its dispatches (KiB for *_SIZE)."""
    cur = _db(path).cursor()
    rows = cur.execute("select kernel_name, grid_size, value from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    agg = collections.defaultdict(list)
    for k, g, v in rows:
        agg[(k, g)].append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
               "SQ_INSTS_VMEM_WR", "SQ_INSTS_SALU", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")


def sq_per_wave(path):
    """Per kernel: SQ counters summed over its dispatches and divided by the
    summed SQ_WAVES (instructions or cycles per wave)."""
    cur = _db(path).cursor()
    rows = cur.execute("select kernel_name, counter_name, sum(value) from counters_collection "
                       "group by kernel_name, counter_name").fetchall()
    tot = collections.defaultdict(dict)
    for k, c, v in rows:
        tot[k][c] = v
    out = {}
    for k, cs in tot.items():
        waves = cs.get("SQ_WAVES")
        if waves:
            out[k] = {c: cs[c] / waves for c in cs if c != "SQ_WAVES"}
            out[k]["waves"] = waves
    return out


def _pooled(means, pred):
    tot, cnt = 0.0, 0
    for (k, _g), (m, c) in means.items():
        if pred(k):
            tot += m * c
            cnt += c
    return (tot / cnt if cnt else None), cnt


def summarize(a):
    trace = kernel_stats(a.trace)
    fetch = counter_means(a.fetch, "FETCH_SIZE")
    write = counter_means(a.write, "WRITE_SIZE")
    is_pass = lambda k: k.startswith(PASS_PREFIX)
    is_copy = lambda k: k.startswith(COPY_NAME)
    copy_f, _ = _pooled(fetch, is_copy)
    copy_w, _ = _pooled(write, is_copy)
    pass_f, nf = _pooled(fetch, is_pass)
    pass_w, nw = _pooled(write, is_pass)
    copy_kib = a.copy_bytes / 1024.0
    f_factor = copy_kib / copy_f if copy_f else None
    w_factor = copy_kib / copy_w if copy_w else None
    traffic = None
    if None not in (pass_f, pass_w, f_factor, w_factor):
        traffic = (pass_f * f_factor + pass_w * w_factor) * 1024.0
    pass_trace = [t for t in trace if is_pass(t["name"])]
    calls = sum(t["calls"] for t in pass_trace)
    avg_ns = sum(t["total_ns"] for t in pass_trace) / calls if calls else None
    # per pass-kernel instance: duration and scaled counter bytes per launch;
    # the dominant kernel is the one with the longest average launch
    per_kernel = {}
    for t in pass_trace:
        fk = [v for (k, _g), v in fetch.items() if k == t["name"]]
        wk = [v for (k, _g), v in write.items() if k == t["name"]]
        fm = sum(m * c for m, c in fk) / max(1, sum(c for _m, c in fk)) if fk else None
        wm = sum(m * c for m, c in wk) / max(1, sum(c for _m, c in wk)) if wk else None
        tb = None
        if None not in (fm, wm, f_factor, w_factor):
            tb = (fm * f_factor + wm * w_factor) * 1024.0
        per_kernel[t["name"]] = {"avg_ns": t["avg_ns"], "calls": t["calls"], "fetch_kib": fm,
                                 "write_kib": wm, "traffic_bytes_per_launch": tb}
    dominant = max(per_kernel, key=lambda k: per_kernel[k]["avg_ns"]) if per_kernel else None
    bench = None
    if a.bench_json and os.path.exists(a.bench_json):
        for line in open(a.bench_json):
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                bench = json.loads(line)
    alg = None
    if bench:
        alg = bench.get("roofline", {}).get("algorithmic_bytes_per_launch")
    block = {
        "source_digest": source_digest(),
        "workload": bench["config"] if bench else None,
        "pass_kernel_avg_ns": avg_ns,
        "pass_fetch_kib": pass_f,
        "pass_write_kib": pass_w,
        "copy_bytes_each_way": a.copy_bytes,
        "copy_fetch_kib": copy_f,
        "copy_write_kib": copy_w,
        "fetch_factor": f_factor,
        "write_factor": w_factor,
        "pass_traffic_bytes_per_launch": traffic,
        "kernels": per_kernel,
        "dominant_kernel": dominant,
        "dominant_avg_ns": per_kernel[dominant]["avg_ns"] if dominant else None,
        "dominant_traffic_bytes_per_launch":
            per_kernel[dominant]["traffic_bytes_per_launch"] if dominant else None,
        "algorithmic_bytes_per_launch": alg,
        "dominant_frac_of_8tbs": (alg / per_kernel[dominant]["avg_ns"] / 8000.0
                                  if (alg and dominant) else None),
    }
    out = []
    out.append(f"# {a.title}\n")
    out.append("Commands (run from the repository root, after `cd /tmp && export TMPDIR=/tmp`):\n")
    for label, c in (("kernel trace", a.cmd_trace), ("FETCH_SIZE", a.cmd_fetch),
                     ("WRITE_SIZE", a.cmd_write)):
        out.append(f"* {label}: `{c}`")
    out.append("")
    out.append("## Kernel trace (`--kernel-trace --stats`)\n")
    out.append("| kernel | calls | avg µs | min µs | max µs | VGPR | AGPR | scratch B | LDS B |")
    out.append("|---|---|---|---|---|---|---|---|---|")
    for t in trace:
        out.append(f"| `{t['name'][:90]}` | {t['calls']} | {t['avg_ns'] / 1e3:.1f} | "
                   f"{t['min_ns'] / 1e3:.1f} | {t['max_ns'] / 1e3:.1f} | {t['vgpr']} | "
                   f"{t['agpr']} | {t['scratch']} | {t['lds']} |")
    out.append("")
    out.append("## HBM counters (KiB per dispatch, mean over dispatches)\n")
    out.append("| kernel | grid | FETCH_SIZE | WRITE_SIZE | dispatches |")
    out.append("|---|---|---|---|---|")
    for key in sorted(set(fetch) | set(write)):
        fm = fetch.get(key, (float("nan"), 0))
        wm = write.get(key, (float("nan"), 0))
        out.append(f"| `{key[0][:90]}` | {key[1]} | {fm[0]:.1f} | {wm[0]:.1f} | {fm[1]}/{wm[1]} |")
    out.append("")
    out.append("## Scaling against the plain copy\n")
    if f_factor and w_factor:
        out.append(f"The device copy moves {a.copy_bytes} bytes each way "
                   f"({copy_kib:.0f} KiB). FETCH_SIZE reads {copy_f:.1f} KiB "
                   f"(factor {f_factor:.4f}); WRITE_SIZE reads {copy_w:.1f} KiB "
                   f"(factor {w_factor:.4f}).")
    if traffic:
        out.append(f"Pass kernel, scaled: {traffic / 2**30:.4f} GiB per launch "
                   f"({nf} / {nw} dispatches counted).")
    if dominant:
        d = per_kernel[dominant]
        line = (f"Dominant kernel (longest average launch): `{dominant[:90]}`, "
                f"{d['avg_ns'] / 1e3:.1f} µs")
        if alg:
            line += (f"; {alg} algorithmic bytes per launch, {alg / d['avg_ns']:.1f} GB/s, "
                     f"{alg / d['avg_ns'] / 8000.0:.3f} of 8 TB/s")
        if d["traffic_bytes_per_launch"]:
            line += f"; counters {d['traffic_bytes_per_launch'] / 2**30:.4f} GiB per launch"
        out.append(line + ".")
    if bench:
        r = bench.get("roofline", {})
        pm = bench.get("pass_ms") or []
        out.append("")
        out.append(f"Bench line of the traced run: {bench['ms_per_step']:.4f} ms per step; "
                   f"HIP-event pass times {', '.join(f'{m:.4f}' for m in pm)} ms; "
                   f"roofline frac {r.get('frac', float('nan')):.3f} ({r.get('kernel', '')}).")
    out.append("")
    out.append("VGPR and AGPR as rocprofv3 reports them: on gfx950 the figure is half the "
               "registers the compiler allocates (its resource report: 157 for a 'VGPR 80' "
               "here).")
    if getattr(a, "sq", None):
        sq = sq_per_wave(a.sq)
        cols = [c for c in SQ_COUNTERS if c != "SQ_WAVES"]
        out.append("")
        out.append("## SQ counters per wave\n")
        out.append(f"* SQ counters: `{a.cmd_sq}`\n")
        out.append("| kernel | waves | " + " | ".join(c[3:] for c in cols) + " |")
        out.append("|---|---|" + "---|" * len(cols))
        for k in sorted(sq):
            if not is_pass(k):
                continue
            v = sq[k]
            out.append(f"| `{k[:90]}` | {v['waves']:.0f} | "
                       + " | ".join(f"{v.get(c, float('nan')):.0f}" for c in cols) + " |")
        out.append("")
        out.append("Instruction counts are per wave. SQ_WAVE_CYCLES and SQ_WAIT_INST_ANY are "
                   "summed over waves by the hardware, in its own cycle units, and divided "
                   "the same way.")
    out.append("")
    out.append("## Machine-readable\n")
    out.append("```json")
    out.append(json.dumps(block, indent=1))
    out.append("```")
    return "\n".join(out) + "\n"


def _load_block(md_path, config):
    """The summary's JSON block, or None when the summary is missing, was
    taken on other sources, or on another workload."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    start = text.find("```json")
    if start < 0:
        return None
    end = text.find("```", start + 7)
    try:
        block = json.loads(text[start + 7:end])
    except ValueError:
        return None
    if block.get("source_digest") != source_digest():
        return None
    w = block.get("workload") or {}
    for key in ("n", "cutoff", "pass_bits", "kernel_config", "workload"):
        if w.get(key) != config.get(key):
            return None
    return block


def load_traffic(md_path, config, kernel=None):
    """Scaled HBM bytes per launch of one pass kernel instance (`kernel`, a
    name such as "k_fused_pass2<float, 5, 4, true, true>"), or pooled over
    every pass launch when kernel is None; None when the summary does not
    apply (see _load_block) or lacks that kernel."""
    block = _load_block(md_path, config)
    if block is None:
        return None
    if kernel is None:
        return block.get("pass_traffic_bytes_per_launch")
    for name, v in (block.get("kernels") or {}).items():
        if ("qft::" + kernel + "(") in name:
            return v.get("traffic_bytes_per_launch")
    return None


def load_plan_traffic(md_path, config):
    """Scaled HBM bytes of one whole transform (mean per pass launch times
    the plan's passes), or None."""
    block = _load_block(md_path, config)
    if block is None or not block.get("pass_traffic_bytes_per_launch"):
        return None
    return block["pass_traffic_bytes_per_launch"] * config.get("passes", 0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--cmd-trace", required=True)
    ap.add_argument("--cmd-fetch", required=True)
    ap.add_argument("--cmd-write", required=True)
    ap.add_argument("--bench-json", default=None)
    ap.add_argument("--sq", default=None, help="rocprofv3 --pmc run of the SQ counters")
    ap.add_argument("--cmd-sq", default="")
    ap.add_argument("--title", default="Fused pass kernel, exact QFT n = 28 complex64")
    print(summarize(ap.parse_args()), end="")


if __name__ == "__main__":
    main()
