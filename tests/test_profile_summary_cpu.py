"""The rocprofv3 summary tool and the traffic lookup that bench.py does with it.

Synthetic result databases with the two views the tool reads (top_kernels,
counters_collection) stand in for rocprofv3 output.
"""

import argparse
import json
import sqlite3

from paper_2606_18981_amd import profile_summary as PS

PASS = "void qft::k_fused_pass<float, 5>(qft::PassDesc, qft::cplx<float> const*, qft::cplx<float>*)"
COPY = "__amd_rocclr_copyBuffer"
GIB = 1 << 30


def _trace_db(path):
    db = sqlite3.connect(path)
    db.execute("create table kernels (name, duration, vgpr_count, accum_vgpr_count, "
               "scratch_size, lds_size)")
    for d in (1.0e6, 1.1e6, 1.2e6, 1.0e6, 1.1e6, 1.2e6):
        db.execute("insert into kernels values (?,?,?,?,?,?)", (PASS, d, 224, 0, 0, 65536))
    for d in (0.88e6, 0.9e6, 0.92e6, 0.9e6):
        db.execute("insert into kernels values (?,?,?,?,?,?)", (COPY, d, 16, 0, 0, 0))
    db.commit()


def _pmc_db(path, counter, pass_kib, copy_kib):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (kernel_name, grid_size, counter_name, value)")
    for _ in range(3):
        db.execute("insert into counters_collection values (?,?,?,?)",
                   (PASS, 1 << 20, counter, pass_kib))
        db.execute("insert into counters_collection values (?,?,?,?)",
                   (COPY, 1 << 17, counter, copy_kib))
    db.commit()


def test_summary_scales_counters_by_the_copy_and_round_trips(tmp_path):
    _trace_db(tmp_path / "trace.db")
    # FETCH reads half of the true bytes on both kernels, WRITE reads them exactly
    _pmc_db(tmp_path / "fetch.db", "FETCH_SIZE", GIB / 1024 / 2 * 1.01, GIB / 1024 / 2)
    _pmc_db(tmp_path / "write.db", "WRITE_SIZE", GIB / 1024, GIB / 1024)
    config = {"workload": "w", "n": 28, "cutoff": -1, "pass_bits": [9, 10, 9],
              "kernel_config": {"tile_log2": 13}}
    bench = tmp_path / "bench.log"
    bench.write_text("[bench] noise\n" + json.dumps(
        {"metric": "m", "ms_per_step": 3.3, "config": config,
         "roofline": {"algorithmic_bytes_per_launch": 2 * GIB, "achieved": 1950.0}}) + "\n")
    a = argparse.Namespace(trace=str(tmp_path / "trace.db"), fetch=str(tmp_path / "fetch.db"),
                           write=str(tmp_path / "write.db"), copy_bytes=GIB,
                           cmd_trace="t", cmd_fetch="f", cmd_write="w",
                           bench_json=str(bench), title="x")
    md = PS.summarize(a)
    assert "factor 2.0000" in md and "factor 1.0000" in md
    assert "| 6 | 1100.0 | 1000.0 | 1200.0 | 224 |" in md
    path = tmp_path / "s.md"
    path.write_text(md)
    traffic = PS.load_traffic(str(path), config)
    assert abs(traffic - (1.01 * GIB + GIB)) < 1.0
    # the one pass kernel instance is the dominant one
    assert abs(PS.load_traffic(str(path), config, "k_fused_pass<float, 5>")
               - (1.01 * GIB + GIB)) < 1.0
    assert PS.load_traffic(str(path), config, "k_fused_pass2<float, 5, 4, true, true>") is None
    assert abs(PS.load_plan_traffic(str(path), dict(config, passes=3))
               - 3 * (1.01 * GIB + GIB)) < 4.0
    assert "Dominant kernel (longest average launch)" in md
    # another workload or other kernel sources: no traffic figure
    assert PS.load_traffic(str(path), dict(config, pass_bits=[10, 9, 9])) is None
    assert PS.load_traffic(str(path).replace("s.md", "none.md"), config) is None
    path.write_text(md.replace(PS.source_digest(), "0" * 16))
    assert PS.load_traffic(str(path), config) is None


def test_sq_counters_per_wave(tmp_path):
    db = sqlite3.connect(tmp_path / "sq.db")
    db.execute("create table counters_collection (kernel_name, grid_size, counter_name, value)")
    for _ in range(2):  # two dispatches of 100 waves each
        for c, v in (("SQ_WAVES", 100), ("SQ_INSTS_VALU", 170000), ("SQ_INSTS_LDS", 9000),
                     ("SQ_WAVE_CYCLES", 5.0e6)):
            db.execute("insert into counters_collection values (?,?,?,?)", (PASS, 1 << 20, c, v))
    db.commit()
    sq = PS.sq_per_wave(str(tmp_path / "sq.db"))
    assert sq[PASS]["waves"] == 200
    assert sq[PASS]["SQ_INSTS_VALU"] == 1700
    assert sq[PASS]["SQ_INSTS_LDS"] == 90
    assert sq[PASS]["SQ_WAVE_CYCLES"] == 50000
