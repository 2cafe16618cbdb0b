"""Host-side checks of libqft.so that need no GPU.

* the library loads and exports every function declared in include/*.h;
* argument validation and error codes of the host planner;
* pass partition: every qubit applied exactly once, in descending order;
* gate counts before fusion (the paper's aggregate counters);
* twiddle tables against FP64 numpy within the dtype's rounding;
* a test-only numpy replay of the fused kernel over the planner's maps
  (tests/plan_emulator.py) against the oracle, for many configurations.
"""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2606_18981_amd import inputs as I
from paper_2606_18981_amd import qft as Q

import plan_emulator as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(qft_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert "qft_plan" in names and "qft_execute" in names and "qft_destroy" in names
    lib = ctypes.CDLL(Q.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_descriptor_layout_matches():
    assert E.desc_size_matches()


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(n=32), dict(n=-3), dict(norm=7), dict(layout=0x80), dict(layout=0x40),
])
def test_invalid_arguments(bad):
    args = dict(n=10, cutoff=-1, norm=0, layout=0)
    args.update(bad)
    info = Q.PlanInfo()
    rc = Q.lib.qft_plan_describe(args["n"], args["cutoff"], args["norm"], args["layout"],
                                 None, ctypes.byref(info))
    assert rc == Q.QFT_ERR_INVALID
    assert Q.last_error() != ""


def test_invalid_config():
    for cfg in (dict(radix_log2=6), dict(tile_log2=16), dict(tile_log2=12, radix_log2=1)):
        with pytest.raises(Q.QftError) as e:
            Q.describe(16, config=cfg)
        assert e.value.code == Q.QFT_ERR_INVALID


def test_null_plan_is_rejected_without_gpu():
    assert Q.lib.qft_execute(None, None, None) == Q.QFT_ERR_INVALID
    Q.lib.qft_destroy(None)  # NULL-safe
    info = Q.PlanInfo()
    assert Q.lib.qft_plan_info(None, ctypes.byref(info)) == Q.QFT_ERR_INVALID


@pytest.mark.parametrize("n", [1, 2, 7, 10, 13, 14, 20, 22, 24, 26, 28, 30, 31])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("order", ["natural", "bitrev"])
def test_pass_partition_covers_each_qubit_once(n, dtype, order):
    info = Q.describe(n, -1, "unitary", dtype, order)
    P = info.num_passes
    assert 1 <= P <= Q.QFT_MAX_PASSES
    top = n
    for p in range(P):
        lo, m = info.pass_lo[p], info.pass_bits[p]
        assert m >= 1 and lo + m == top  # descending, contiguous
        top = lo
        assert info.pass_reverse[p] == (1 if (order == "natural" and p == P - 1) else 0)
    assert top == 0
    es = 16 if dtype == "c128" else 8
    assert info.state_bytes == es << n
    assert info.hbm_bytes == 2 * P * info.state_bytes
    assert info.workspace_bytes == (info.state_bytes if (order == "natural" and P > 1) else 0)


def test_headline_pass_counts():
    # n = 28 and 30 in three HBM passes for both element sizes (complex128
    # n = 30 reaches 128-byte first-pass rows through its 2^13 tiles; with
    # 2^12 tiles everywhere it takes four); n <= 13 (complex64) or <= 12
    # (complex128) in one
    for dt in ("c64", "c128"):
        assert Q.describe(28, dtype=dt).num_passes == 3
        assert Q.describe(30, dtype=dt).num_passes == 3
    assert list(Q.describe(30, dtype="c128").pass_bits)[:3] == [10, 10, 10]
    narrow = dict(pass_tile_log2=[12, 12, 12, 12])
    assert Q.describe(30, dtype="c128", config=narrow).num_passes == 3  # explicit tiles
    assert Q.describe(31, dtype="c128").num_passes == 4
    assert Q.describe(13, dtype="c64").num_passes == 1
    assert Q.describe(12, dtype="c128").num_passes == 1


@pytest.mark.parametrize("n,k", [(22, 21), (22, 16), (22, 12), (22, 10), (22, 8), (22, 6),
                                 (22, 4), (28, 6), (30, -1), (3, 1)])
def test_gate_counts_before_fusion(n, k):
    info = Q.describe(n, k)
    ref = O.gate_counts(n, k)
    assert (info.gates_h, info.gates_cr, info.gates_swap) == (ref["H"], ref["CR"], ref["SWAP"])
    assert info.cutoff == O.effective_cutoff(n, k)


def test_gate_schedule_description():
    info = Q.describe(10, -1, "unitary", "c128", "natural", "gates")
    assert info.num_passes == 10 + 45 + 5
    info = Q.describe(10, -1, "none", "c128", "bitrev", "gates")
    assert info.num_passes == 10 + 45 + 1  # no swaps, one output scale


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_twiddle_tables(dtype):
    n = 20
    layout = Q.layout_flags(dtype)
    W, tlo, thi, es = E.get_tables(n, -1, "unitary", layout, None)
    # numpy evaluates exp(-2 pi i x / N) with its own ~1 ulp angle rounding
    ulp = 4 * 2.0 ** -52 if dtype == "c128" else 2.0 ** -23
    MI = int(math.log2(W.size)) + 1
    y = np.arange(W.size)
    assert np.max(np.abs(W - np.exp(-2j * np.pi * y / 2 ** MI))) < ulp
    L = int(math.log2(tlo.size))
    x = np.arange(tlo.size)
    assert np.max(np.abs(tlo - np.exp(-2j * np.pi * x / 2 ** n))) < ulp
    x = np.arange(thi.size)
    assert np.max(np.abs(thi - np.exp(-2j * np.pi * (x << L) / 2 ** n))) < ulp
    # exact values at the quarter turns
    assert W[0] == 1 and tlo[0] == 1
    assert thi[thi.size // 4] == -1j and thi[thi.size // 2] == -1


CASES = []
for n in (1, 2, 3, 4, 6, 9, 13, 14, 15, 17):
    for k in (None, 0, 1, 2, 5):
        CASES.append((n, k, "unitary", "c128", "natural", None))
for n in (5, 12, 16):
    for norm in O.NORMS:
        for order in O.ORDERS:
            CASES.append((n, 3, norm, "c64", order, None))
CONFIGS = [
    dict(tile_log2=6, radix_log2=1, spec_log2=2, rev_spec_log2=2),
    dict(tile_log2=7, radix_log2=2, spec_log2=3, rev_spec_log2=1),
    dict(tile_log2=8, radix_log2=3, spec_log2=-1, rev_spec_log2=-1),
    dict(tile_log2=9, radix_log2=5, spec_log2=4, rev_spec_log2=4),
    dict(tile_log2=10, radix_log2=4, spec_log2=5, rev_spec_log2=3),
    dict(tile_log2=11, radix_log2=5, spec_log2=2, rev_spec_log2=3),
]
for cfg in CONFIGS:
    for n, k in ((11, None), (16, 4), (19, 2), (20, None)):
        for order in O.ORDERS:
            CASES.append((n, k, "unitary", "c128", order, cfg))


@pytest.mark.parametrize("n,k,norm,dtype,order,cfg", CASES)
def test_emulated_kernel_matches_oracle(n, k, norm, dtype, order, cfg):
    x = I.gaussian(n, 1000 + n)
    cut = -1 if k is None else k
    y = E.emulate(x, n, cut, norm, dtype, order, cfg)
    ref = O.qft_fused_targets(x, k, norm, order)
    tol = 1e-12 if dtype == "c128" else 2e-6
    assert O.rel_l2(y, ref) < tol


@pytest.mark.parametrize("split", [[7, 7, 6], [5, 8, 7], [10, 10], [4, 4, 4, 4, 4]])
def test_explicit_pass_splits(split):
    n = sum(split)
    cfg = dict(tile_log2=12, radix_log2=4, spec_log2=2, rev_spec_log2=2, pass_bits=split)
    info = Q.describe(n, -1, "unitary", "c128", "natural", "fused", cfg)
    assert list(info.pass_bits)[:info.num_passes] == split
    x = I.gaussian(n, 77)
    for k in (None, 3):
        y = E.emulate(x, n, -1 if k is None else k, "unitary", "c128", "natural", cfg)
        assert O.rel_l2(y, O.qft_fused_targets(x, k)) < 1e-12


def test_invalid_pass_splits():
    for split in ([7, 7, 5], [0, 10, 10], [14, 6]):
        with pytest.raises(Q.QftError):
            Q.describe(20, config=dict(tile_log2=12, radix_log2=4, pass_bits=split))


def test_tile_number_order():
    # consecutive tile numbers differ in the non-tile bits nearest the bottom
    # of the written address: ascending input bits in place, descending input
    # bits in the bit-reversing pass
    layout = Q.layout_flags("c64")
    info = Q.describe(28)
    for p in range(info.num_passes):
        d, L = E.get_pass(28, -1, "unitary", layout, None, p)
        free = [E.P(d.free_w)[b] for b in range(d.nfree)]
        assert sorted(free) == (free[::-1] if d.reverse else free)
        assert L[2] == d.ntiles == 1 << d.nfree
    assert info.pass_reverse[info.num_passes - 1] == 1


def test_emulated_three_pass_plan():
    # a three-pass plan at n = 21 (complex64 default tiles) and an AQFT one
    n = 21
    x = I.gaussian(n, 7)
    assert Q.describe(n, dtype="c64").num_passes == 3
    for k in (None, 8):
        y = E.emulate(x, n, -1 if k is None else k, "unitary", "c64", "natural")
        assert O.rel_l2(y, O.qft_fused_targets(x, k)) < 2e-6


INV_CASES = [
    (6, None, "unitary", "c128", "natural", None),
    (12, 4, "none", "c64", "bitrev", None),
    (17, None, "inv_n", "c128", "natural", dict(tile_log2=9, radix_log2=3, spec_log2=2,
                                                 rev_spec_log2=2)),
    (20, 6, "unitary", "c128", "natural", dict(tile_log2=10, radix_log2=4, spec_log2=3,
                                                rev_spec_log2=3)),
]


@pytest.mark.parametrize("n,k,norm,dtype,order,cfg", INV_CASES)
def test_emulated_inverse_matches_oracle(n, k, norm, dtype, order, cfg):
    x = I.gaussian(n, 1500 + n)
    y = E.emulate(x, n, -1 if k is None else k, norm, dtype, order, cfg, inverse=True)
    ref = O.qft_fused_targets(x, k, norm, order, inverse=True)
    assert O.rel_l2(y, ref) < (1e-12 if dtype == "c128" else 2e-6)


def test_inverse_descriptor_flags():
    layout = Q.layout_flags("c64", inverse=True)
    info = Q.describe(28, inverse=True)
    assert info.layout & Q.QFT_INVERSE
    P = info.num_passes
    for p in range(P):
        d, _ = E.get_pass(28, -1, "unitary", layout, None, p)
        assert d.conj_in == (1 if p == 0 else 0) and d.conj_out == (1 if p == P - 1 else 0)
    d, _ = E.get_pass(28, -1, "unitary", Q.layout_flags("c64"), None, 0)
    assert d.conj_in == 0 and d.conj_out == 0
    # one-pass plan: both on the same pass
    d, _ = E.get_pass(10, -1, "unitary", layout, None, 0)
    assert d.conj_in == 1 and d.conj_out == 1


def test_nontemporal_rule():
    # streaming access on passes whose tiles read whole 128-byte lines, and
    # only when the state is larger than the 256 MB Infinity Cache
    def nts(n, dtype="c64", cfg=None):
        lay = Q.layout_flags(dtype)
        P = Q.describe(n, dtype=dtype, config=cfg).num_passes
        return [E.get_pass(n, -1, "unitary", lay, cfg, p)[0].nt for p in range(P)]
    assert nts(28) == [1, 1, 1]        # 256 B rows, 128 B rows (2^14 tiles), contiguous
    assert nts(27) == [1, 0, 1]        # 256 B rows, 64 B rows, contiguous
    assert nts(27, "c128") == [1, 1, 1]   # 2^13 tiles: 128 B middle rows
    assert nts(25, "c128") == [1, 1, 1]   # 2^13 tiles: 128 B middle rows
    assert nts(24) == [0, 0, 0]        # 128 MiB state: stays cached
    assert nts(25) == [1, 0, 1]        # 256 MiB
    assert nts(24, "c128") == [1, 0, 1]
    assert nts(24, cfg=dict(nontemporal=2)) == [1, 0, 1]
    assert nts(28, cfg=dict(nontemporal=1)) == [0, 0, 0]


@pytest.mark.parametrize("n,k,dtype", [(28, None, "c64"), (27, None, "c128"), (24, 8, "c64"),
                                       (21, 6, "c128"), (21, 3, "c128")])
def test_group_factor_tables(n, k, dtype):
    # every pass of the specialised two-group shape gets a per-thread table
    # holding exactly the internal-table entries its first group reads
    lay = Q.layout_flags(dtype)
    cut = -1 if k is None else k
    info = Q.describe(n, cut, dtype=dtype)
    W = E.get_tables(n, cut, "unitary", lay, None)[0]
    image, dt = E.get_table_image(n, cut, "unitary", lay, None)
    checked = 0
    for p in range(info.num_passes):
        d, launch = E.get_pass(n, cut, "unitary", lay, None, p)
        assert bool(d.gtab) == bool(info.pass_kernel[p])
        checked += E.check_group_table(d, launch, image, dt, W)
    assert checked == sum(1 for p in range(info.num_passes) if info.pass_kernel[p])
    # radix 32 needs k >= 4 (a register group spans at most k + 1 qubits)
    assert (checked > 0) == (k is None or k >= 4)


def test_split_exchange_lds():
    # complex64 two-group passes exchange real and imaginary parts in turn
    # through half the tile; complex128 ones use the whole tile, except the
    # lean 2^13-tile form (256 threads), which splits too
    for n, dtype, es in ((27, "c64", 8), (27, "c128", 16), (24, "c128", 16)):
        lay = Q.layout_flags(dtype)
        info = Q.describe(n, dtype=dtype)
        for p in range(info.num_passes):
            d, launch = E.get_pass(n, -1, "unitary", lay, None, p)
            assert info.pass_kernel[p]
            full = (1 << d.T) * es
            half = dtype == "c64" or launch[0] == 256
            assert launch[1] == (full // 2 if half else full), (n, dtype, p)


def test_wide_first_pass():
    """A first pass that would hold fewer than 4 row bits (64-byte complex64
    rows) takes one more tile bit: n = 30 at the default tiles, and a small
    plan with 2^10 tiles, checked by emulation."""
    # n = 28..30 complex64 passes get 2^14 tiles anyway (wide high passes);
    # the rule shows with those turned off by explicit 2^13 pass tiles
    info = Q.describe(30, dtype="c64", config=dict(pass_tile_log2=[0, 13, 13]))
    assert list(info.pass_bits)[:3] == [10, 10, 10]
    assert list(info.pass_spec)[:3] == [4, 3, 3]
    for n, spec in ((28, [5, 4, 4]), (29, [5, 3, 4]), (30, [4, 4, 4])):
        assert list(Q.describe(n, dtype="c64").pass_spec)[:3] == spec
    assert list(Q.describe(29, dtype="c128").pass_spec)[:3] == [4, 3, 3]  # 2^13 tiles
    cfg = dict(tile_log2=10, radix_log2=4, spec_log2=3, rev_spec_log2=3)
    n = 21
    info = Q.describe(n, -1, "unitary", "c64", "natural", "fused", cfg)
    assert list(info.pass_bits)[:3] == [7, 7, 7]
    assert list(info.pass_spec)[:3] == [4, 3, 3]
    x = I.gaussian(n, 21)
    for k in (None, 5):
        y = E.emulate(x, n, -1 if k is None else k, "unitary", "c64", "natural", cfg)
        assert O.rel_l2(y, O.qft_fused_targets(x, k)) < 2e-6


def test_four_pass_split():
    """With four or more passes the bit-reversing last pass keeps 4 spectator
    bits, the middle passes take the rounded-up share of the rest and the
    first pass what remains; three-pass plans keep wide middle passes."""
    assert list(Q.describe(31, dtype="c64").pass_bits)[:4] == [6, 8, 8, 9]
    assert list(Q.describe(31, dtype="c128").pass_bits)[:4] == [7, 8, 8, 8]
    for dtype in ("c64", "c128"):
        info = Q.describe(31, dtype=dtype)
        assert info.num_passes == 4 and info.pass_spec[3] == 4
    assert list(Q.describe(28, dtype="c64").pass_bits)[:3] == [9, 10, 9]
    # every split of a small-tile configuration still covers each qubit once
    cfg = dict(tile_log2=9, radix_log2=5, spec_log2=4, rev_spec_log2=4)
    for n in range(10, 26):
        info = Q.describe(n, -1, "unitary", "c64", "natural", "fused", cfg)
        bits = list(info.pass_bits)[:info.num_passes]
        assert sum(bits) == n and min(bits) >= 1


def test_three_pass_last_pass_rule():
    """Three-pass plans give the bit-reversing last pass T - 4 bits where the
    first pass keeps at least 6 bits and 256-byte rows (128-byte rows through
    the wider complex64 first-pass tile), and otherwise split the outer
    passes evenly."""
    expect = {("c64", 24): [7, 10, 7], ("c64", 25): [6, 10, 9], ("c64", 26): [7, 10, 9],
              ("c64", 27): [8, 10, 9], ("c64", 28): [9, 10, 9], ("c64", 29): [9, 11, 9],
              ("c128", 24): [6, 10, 8], ("c128", 26): [8, 10, 8], ("c128", 27): [8, 10, 9],
              ("c128", 28): [9, 10, 9]}
    for (dtype, n), bits in expect.items():
        info = Q.describe(n, dtype=dtype)
        assert list(info.pass_bits)[:info.num_passes] == bits, (dtype, n)
    # bit-reversed plans have no reversing pass: the even split stays
    assert list(Q.describe(26, dtype="c64", order="bitrev").pass_bits)[:3] != [7, 10, 9]


def test_three_group_middle_pass_rule():
    """A complex64 three-pass plan whose first pass would hold T - 3 bits and
    T - 4 after giving one to the middle pass (n = 29) runs an 11-bit middle
    pass on the three-group kernel; other sizes, complex128 and bit-reversed
    plans keep 10-bit middles."""
    info = Q.describe(29, dtype="c64")
    assert list(info.pass_bits)[:3] == [9, 11, 9]
    assert info.pass_kernel[1] == 10 + 1 + 3 + 0  # below-pass diagonal, s = 1
    assert list(Q.describe(30, dtype="c64").pass_bits)[:3] == [10, 10, 10]
    for n in list(range(21, 29)) + [30]:
        info = Q.describe(n, dtype="c64")
        assert max(info.pass_kernel[p] for p in range(info.num_passes)) <= 10
    assert max(Q.describe(29, dtype="c128").pass_bits) == 10
    assert list(Q.describe(29, dtype="c64", order="bitrev").pass_bits)[:3] == [9, 10, 10]
    # an AQFT whose radix drops below 32 keeps the two-group split
    assert list(Q.describe(30, 3, dtype="c64").pass_bits)[:3] == [10, 10, 10]


def test_wide_high_pass_tiles():
    """Three-pass plans of 2^28..2^30 complex64 or 2^25..2^30 complex128
    elements give every pass below which other qubits lie one more tile bit
    (2^14 complex64 tiles of 512 threads, 2^13 complex128 of 256: the lean
    kernels), and the last pass too where its rows would otherwise be
    shorter than 128 bytes; other sizes keep 2^13 (complex128 2^12).
    Bit-reversed-order plans widen their high passes only: their last pass
    stores whole tiles in input order."""
    lay = Q.layout_flags("c64")
    expect = {28: [14, 14, 13], 29: [14, 14, 13], 30: [14, 14, 14]}
    for n, tiles in expect.items():
        info = Q.describe(n, dtype="c64")
        for p in range(3):
            d, launch = E.get_pass(n, -1, "unitary", lay, None, p)
            assert d.T == tiles[p] and launch[0] == 1 << (tiles[p] - 5), (n, p)
            assert info.pass_spec[p] == tiles[p] - info.pass_bits[p]
    for n in (24, 25, 26, 27, 31):
        info = Q.describe(n, dtype="c64")
        for p in range(info.num_passes):
            d, _ = E.get_pass(n, -1, "unitary", lay, None, p)
            assert d.T <= 13 or (n == 31 and p == 0), (n, p, d.T)
    c128 = {24: [12, 12, 12], 25: [13, 13, 12], 26: [13, 13, 12], 28: [13, 13, 12],
            29: [13, 13, 13], 30: [13, 13, 13]}
    for n, tiles in c128.items():
        for p in range(3):
            d, launch = E.get_pass(n, -1, "unitary", Q.layout_flags("c128"), None, p)
            assert d.T == tiles[p], (n, p)
            assert launch[0] == 1 << (tiles[p] - 5)
    for n, tiles in {28: [14, 14, 13], 30: [14, 14, 13]}.items():
        for p in range(3):
            d, _ = E.get_pass(n, -1, "unitary", Q.layout_flags("c64", "bitrev"), None, p)
            assert d.T == tiles[p], (n, p, d.T)


def test_pass_tile_config():
    """pass_tile_log2 sets each pass's tile (its spectators are tile minus
    qubits); out-of-range entries are refused; the plan still computes the
    transform (emulated)."""
    cfg = dict(tile_log2=10, radix_log2=4, spec_log2=2, rev_spec_log2=2, pass_bits=[6, 7, 5],
               pass_tile_log2=[11, 9, 12])
    info = Q.describe(18, -1, "unitary", "c128", "natural", "fused", cfg)
    assert list(info.pass_spec)[:3] == [5, 2, 7]
    x = I.gaussian(18, 18)
    for k in (None, 5):
        y = E.emulate(x, 18, -1 if k is None else k, "unitary", "c128", "natural", cfg)
        assert O.rel_l2(y, O.qft_fused_targets(x, k)) < 1e-12
    for bad in ([5, 13, 13], [16, 13, 13], [-1, 0, 0]):
        with pytest.raises(Q.QftError):
            Q.describe(18, config=dict(pass_bits=[6, 7, 5], pass_tile_log2=bad))


def test_one_pass_radix():
    """One-pass plans take the fewest register groups, then the most
    threads, unless the configuration names a radix."""
    for dtype in ("c64", "c128"):
        lay = Q.layout_flags(dtype)
        got = {n: E.get_pass(n, -1, "unitary", lay, None, 0)[0].r for n in (9, 10, 11, 12, 13)}
        assert got == {9: 5, 10: 5, 11: 4, 12: 4, 13: 5}, (dtype, got)
        assert E.get_pass(12, -1, "unitary", lay, dict(radix_log2=5), 0)[0].r == 5


# Three-group passes (10 + s qubits, s = 1..3): groups 0 and 1 of radix 32,
# the last group reached by cross-lane swaps.  Splits put such a pass first
# (below-pass diagonal, input norm), in the middle, and last (bit-reversed
# stores); complex64 tiles of 2^13 and complex128 tiles of 2^12.
THREE_GROUP = [
    ("c64", [3, 11, 4]), ("c64", [2, 12, 4]), ("c64", [2, 13, 3]), ("c64", [11, 4, 3]),
    ("c64", [4, 3, 11]), ("c64", [5, 13]), ("c128", [4, 11, 3]), ("c128", [3, 12, 3]),
    ("c128", [3, 3, 12]),
]


def _three_group_cfg(dtype, split):
    c64 = dtype == "c64"
    return dict(tile_log2=13 if c64 else 12, radix_log2=5, spec_log2=3 if c64 else 2,
                rev_spec_log2=3 if c64 else 2, pass_bits=split)


@pytest.mark.parametrize("dtype,split", THREE_GROUP)
def test_three_group_pass_maps_and_tables(dtype, split):
    n = sum(split)
    cfg = _three_group_cfg(dtype, split)
    lay = Q.layout_flags(dtype)
    info = Q.describe(n, -1, "unitary", dtype, "natural", "fused", cfg)
    W = E.get_tables(n, -1, "unitary", lay, cfg)[0]
    image, dt = E.get_table_image(n, -1, "unitary", lay, cfg)
    for p in range(info.num_passes):
        d, launch = E.get_pass(n, -1, "unitary", lay, cfg, p)
        m = split[p]
        if m > 10:
            s = m - 10
            assert d.lane_swap == s
            assert info.pass_kernel[p] == 10 + 1 + (3 if d.ext_tw else 0) + (s - 1)
            assert E.check_lane_swap(d, launch)
            assert E.check_group_table(d, launch, image, dt, W, group=0)
            assert E.check_group_table(d, launch, image, dt, W, group=1)
            # the exchange between groups 0 and 1 still uses the half-tile
            # LDS area in complex64
            assert launch[1] == (1 << d.T) * (4 if dtype == "c64" else 16)
        else:
            assert d.lane_swap == 0 and not d.gtab1


@pytest.mark.parametrize("dtype,split", THREE_GROUP)
def test_emulated_three_group_passes(dtype, split):
    n = sum(split)
    cfg = _three_group_cfg(dtype, split)
    x = I.gaussian(n, 2200 + n)
    tol = 1e-12 if dtype == "c128" else 2e-6
    y = E.emulate(x, n, -1, "unitary", dtype, "natural", cfg)
    assert O.rel_l2(y, O.qft_fused_targets(x, None, "unitary", "natural")) < tol
    y = E.emulate(x, n, 6, "unitary", dtype, "bitrev", cfg)
    assert O.rel_l2(y, O.qft_fused_targets(x, 6, "unitary", "bitrev")) < tol
    y = E.emulate(x, n, -1, "none", dtype, "natural", cfg, inverse=True)
    assert O.rel_l2(y, O.qft_fused_targets(x, None, "none", "natural", inverse=True)) < tol


# ---- the comparison folded into the last pass -------------------------------

@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("order", ["natural", "bitrev"])
@pytest.mark.parametrize("inverse", [False, True])
def test_last_pass_can_take_the_comparison(dtype, order, inverse):
    # qft_execute_compare compares in the last pass: that pass must have no
    # below-pass diagonal (no controls lie below qubit 0) and must write the
    # caller's array, for every default plan and for explicit splits
    lay = Q.layout_flags(dtype, order, "fused", inverse)
    cases = [(n, None) for n in range(1, 32)]
    cases += [(sum(s), cfg) for s, cfg in (
        ([7, 6, 11], dict(tile_log2=13, radix_log2=5, spec_log2=3, rev_spec_log2=3,
                          pass_bits=[7, 6, 11])),
        ([6, 10, 8], dict(tile_log2=13, radix_log2=5, spec_log2=3, rev_spec_log2=3,
                          pass_bits=[6, 10, 8], pass_tile_log2=[14, 14, 14])),
        ([6, 6], dict(tile_log2=10, radix_log2=3)))]
    for n, cfg in cases:
        if cfg and dtype == "c128" and cfg.get("pass_tile_log2"):
            continue
        for k in (-1, max(0, n // 3)):
            info = Q.describe(n, k, "unitary", dtype, order, "fused", cfg, inverse=inverse)
            last = info.num_passes - 1
            assert info.pass_lo[last] == 0
            d, launch = E.get_pass(n, k, "unitary", lay, cfg, last)
            assert d.ext_tw == 0, (n, k, cfg)
            assert launch[4] == 0, (n, k, cfg)  # out_ws
            assert not d.cmp_ref and not d.cmp_part


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_bitrev_last_pass_stores_rows(dtype):
    # the last pass of a bit-reversed-order plan writes in input order, and
    # its pass bit 0 is global bit 0: its store map must still put the lowest
    # global bits on the lanes (contiguous rows), through an exchange-only
    # register group when the last radix group holds them in registers
    lay = Q.layout_flags(dtype, "bitrev", "fused")
    for n in range(14, 32):
        info = Q.describe(n, -1, "unitary", dtype, "bitrev")
        last = info.num_passes - 1
        d, launch = E.get_pass(n, -1, "unitary", lay, None, last)
        lanes = E.P(d.st_thr_w)[: d.T - d.r]
        assert lanes[:3] == [0, 1, 2], (n, lanes)
        assert d.grp[d.ngroups - 1].nst == 0
        if d.m <= 10:
            # the compile-time two-group kernel with the store exchange runs
            # it, its group-0 factors from the planner's per-thread table
            assert d.ngroups == 3
            assert info.pass_kernel[last] == 16 + d.grp[1].nst, (n, info.pass_kernel[last])
        else:
            # a three-group pass plus the exchange: the generic kernel
            assert d.ngroups == 4 and info.pass_kernel[last] == 0
        if n in (14, 20, 28):
            W = E.get_tables(n, -1, "unitary", lay, None)[0]
            image, dt = E.get_table_image(n, -1, "unitary", lay, None)
            assert E.check_group_table(d, launch, image, dt, W, group=0)
