"""Tuning-table bookkeeping (CPU only: no device timing)."""

import pytest

from paper_2606_18981_amd import qft as Q


@pytest.fixture(autouse=True)
def clean_table():
    Q.tune_clear()
    yield
    Q.tune_clear()


def test_insert_lookup_and_plan_uses_entry():
    cfg = dict(tile_log2=11, radix_log2=3, spec_log2=2, rev_spec_log2=2)
    assert Q.tune_lookup(20, -1, "c64") is None
    Q.tune_insert(20, -1, "c64", "natural", cfg, 1.5)
    assert Q.tune_lookup(20, -1, "c64") == cfg
    # a cutoff >= n - 1 is the same shape as exact
    assert Q.tune_lookup(20, 19, "c64") == cfg
    assert Q.tune_lookup(20, 8, "c64") is None
    assert Q.tune_lookup(20, -1, "c128") is None


def test_save_load_roundtrip_and_skips_bad_lines(tmp_path):
    cfg = dict(tile_log2=12, radix_log2=4, spec_log2=3, rev_spec_log2=3)
    Q.tune_insert(24, 10, "c128", "bitrev", cfg, 2.25)
    path = tmp_path / "wisdom.jsonl"
    Q.tune_save(path)
    text = path.read_text()
    assert '"n":24' in text and '"cutoff":10' in text
    with open(path, "a") as f:
        f.write("this is not json\n")
        f.write('{"arch":"gfx000","n":10,"cutoff":9,"layout":0,"tile_log2":9,'
                '"radix_log2":3,"spec_log2":2,"rev_spec_log2":2,"ms":1}\n')
        f.write('{"arch":"gfx950","n":10,"cutoff":9,"layout":0,"tile_log2":99,'
                '"radix_log2":3,"spec_log2":2,"rev_spec_log2":2,"ms":1}\n')
    Q.tune_clear()
    assert Q.tune_load(path) == 1
    assert Q.tune_lookup(24, 10, "c128", "bitrev") == cfg
    assert Q.tune_lookup(10, -1, "c64") is None


def test_insert_rejects_invalid_config():
    with pytest.raises(Q.QftError):
        Q.tune_insert(20, -1, "c64", "natural", dict(tile_log2=20, radix_log2=3,
                                                      spec_log2=2, rev_spec_log2=2))


def test_load_missing_file():
    with pytest.raises(Q.QftError):
        Q.tune_load("/nonexistent/wisdom.jsonl")


def test_tune_table_keeps_pass_tiles():
    # per-pass tile sizes survive a save / load round trip
    Q.tune_clear()
    cfg = dict(tile_log2=13, radix_log2=5, spec_log2=3, rev_spec_log2=3,
               pass_bits=[9, 10, 9], pass_tile_log2=[14, 14, 13])
    Q.tune_insert(28, -1, "c64", "natural", cfg, 2.4)
    import tempfile, os
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "wisdom.jsonl")
        Q.tune_save(path)
        Q.tune_clear()
        assert Q.tune_load(path) == 1
    assert Q.tune_lookup(28, -1, "c64") == cfg
    Q.tune_clear()
