"""Test-only CPU emulation of the fused-pass kernel over the planner's maps.

This is NOT a product path and is never called by the library, smoke() or
bench.py.  It replays, with numpy, what k_fused_pass does for every
(tile, thread, register) of every launch the host planner emits: the same
index deposits, LDS exchanges, butterflies, table twiddles, final diagonal
and output addressing.  Tests use it to check the planner's pass partition
and maps, and the twiddle bookkeeping, against the oracle on a machine
without a GPU.
"""

import ctypes

import numpy as np

from paper_2606_18981_amd import qft as Q


MAX_TILE = 15
MAX_RADIX = 5
MAX_GROUPS = 15


u32 = ctypes.c_uint32
i32 = ctypes.c_int32


class GroupMap(ctypes.Structure):
    _fields_ = [("reg_w", u32 * 2), ("thr_w", u32 * 4), ("jbase", i32), ("nst", i32)]


class PassDesc(ctypes.Structure):
    _fields_ = [
        ("n", i32), ("T", i32), ("r", i32), ("m", i32), ("pbase", i32), ("lo", i32),
        ("ngroups", i32), ("reverse", i32), ("ext_tw", i32), ("aqft", i32), ("k", i32),
        ("nfree", i32), ("MI", i32), ("L", i32), ("xcd_remap", i32),
        ("conj_in", i32), ("conj_out", i32), ("nt", i32), ("lane_swap", i32), ("ntiles", u32),
        ("gpos_w", u32 * 4), ("free_w", u32 * 8),
        ("ld_thr_w", u32 * 4), ("ld_reg_w", u32 * 2),
        ("st_thr_w", u32 * 4), ("st_reg_w", u32 * 2),
        ("grp", GroupMap * MAX_GROUPS),
        ("scale", ctypes.c_double),
        ("tw_int", ctypes.c_void_p), ("tw_lo", ctypes.c_void_p), ("tw_hi", ctypes.c_void_p),
        ("gtab", ctypes.c_void_p),
        ("gtab1", ctypes.c_void_p),
        ("norm_part", ctypes.c_void_p),
        ("cmp_ref", ctypes.c_void_p),
        ("cmp_part", ctypes.c_void_p),
    ]


def P(words):
    """Unpack four 8-bit positions per 32-bit word."""
    out = []
    for w in words:
        for b in range(4):
            out.append((w >> (8 * b)) & 0xFF)
    return out


def desc_size_matches() -> bool:
    return ctypes.sizeof(PassDesc) == Q.lib.qft_debug_pass_desc_size()


def get_pass(n, cutoff, norm, layout, config, p):
    d = PassDesc()
    launch = (ctypes.c_int * 5)()
    c = Q._config(config)
    rc = Q.lib.qft_debug_pass(n, cutoff, Q._norm(norm), layout,
                              ctypes.byref(c) if c is not None else None, p,
                              ctypes.byref(d), ctypes.sizeof(d), launch)
    Q._check(rc)
    return d, list(launch)


def get_tables(n, cutoff, norm, layout, config):
    off = (ctypes.c_size_t * 5)()
    c = Q._config(config)
    cref = ctypes.byref(c) if c is not None else None
    Q._check(Q.lib.qft_debug_tables(n, cutoff, Q._norm(norm), layout, cref, None, 0, off))
    buf = (ctypes.c_uint8 * max(1, off[4]))()
    Q._check(Q.lib.qft_debug_tables(n, cutoff, Q._norm(norm), layout, cref, buf, off[4], off))
    dt = np.complex128 if layout & Q.QFT_C128 else np.complex64
    raw = np.frombuffer(bytes(buf), dtype=np.uint8)
    es = np.dtype(dt).itemsize

    def tab(a, b):
        return raw[a:b].view(dt).astype(np.complex128) if b > a else np.zeros(0, np.complex128)

    return tab(off[0], off[1]), tab(off[1], off[2]), tab(off[2], off[3]), es


def get_table_image(n, cutoff, norm, layout, config):
    """The plan's whole table image as raw bytes, and its element dtype."""
    off = (ctypes.c_size_t * 5)()
    c = Q._config(config)
    cref = ctypes.byref(c) if c is not None else None
    Q._check(Q.lib.qft_debug_tables(n, cutoff, Q._norm(norm), layout, cref, None, 0, off))
    buf = (ctypes.c_uint8 * max(1, off[4]))()
    Q._check(Q.lib.qft_debug_tables(n, cutoff, Q._norm(norm), layout, cref, buf, off[4], off))
    dt = np.complex128 if layout & Q.QFT_C128 else np.complex64
    return np.frombuffer(bytes(buf), dtype=np.uint8), dt


def check_group_table(d, launch, image, dt, W, group=0):
    """The planner's per-thread factor table of register group `group`
    (d.gtab for group 0, d.gtab1 for group 1; each a byte offset in the
    image) must hold, bit for bit, the internal-table entries that the
    group's factors read."""
    off = d.gtab if group == 0 else d.gtab1
    if not off:
        return False
    threads = launch[0]
    RB, TR = d.r, d.T - d.r
    G = d.grp[group]
    es = np.dtype(dt).itemsize
    got = image[off:off + RB * threads * es].view(dt).reshape(RB, threads)
    tid = np.arange(threads, dtype=np.int64)
    e = np.zeros_like(tid)
    for b in range(TR):
        e |= ((tid >> b) & 1) << P(G.thr_w)[b]
    u = (e >> d.pbase) & ((1 << G.jbase) - 1)
    for q in range(RB):
        if q >= G.nst:
            assert np.all(got[q] == 1), "unused factor slots hold 1"
            continue
        jl = G.jbase + q
        clear = max(0, jl - d.k) if d.aqft else 0
        x = np.zeros_like(u) if clear >= G.jbase else (u >> clear) << clear
        want = W[x << (d.MI - 1 - jl)].astype(dt)
        assert np.array_equal(got[q], want), f"group {group} table row {q} differs"
    return True


def check_lane_swap(d, launch):
    """A three-group pass's last map must be the middle map with register bit
    q and lane bit 5 - q traded (q < s), as the kernel's cross-lane swaps do,
    and register bits 0..s-1 of the last map must hold pass bits 0..s-1."""
    s = d.lane_swap
    if not s:
        return False
    TR = d.T - d.r
    assert TR >= 6 and d.ngroups == 3 and d.m == 10 + s
    g1, g2 = d.grp[1], d.grp[2]
    r1, t1 = P(g1.reg_w)[:d.r], P(g1.thr_w)[:TR]
    r2, t2 = P(g2.reg_w)[:d.r], P(g2.thr_w)[:TR]
    for q in range(d.r):
        want = t1[5 - q] if q < s else r1[q]
        assert r2[q] == want, "last group's register map is not the swapped middle map"
    for b in range(TR):
        want = r1[5 - b] if 5 - s < b <= 5 else t1[b]
        assert t2[b] == want, "last group's thread map is not the swapped middle map"
    for q in range(s):
        assert r2[q] == d.pbase + q, "register bit q of the last group must be pass bit q"
    return True


def _swizzle(e, c128):
    sw = 3 if c128 else 4
    h = (e >> sw) ^ (e >> (2 * sw)) ^ (e >> (3 * sw)) ^ (e >> (4 * sw))
    return e ^ (h & ((1 << sw) - 1))


def _bitrev(x, n):
    r = np.zeros_like(x)
    for b in range(n):
        r |= ((x >> b) & 1) << (n - 1 - b)
    return r


def run_pass(d, launch, src, tables, c128, check=True):
    """Emulate one launch; returns (output indices, values) for all tiles."""
    W, tlo, thi, _ = tables
    T, RB = d.T, d.r
    R = 1 << RB
    TR = T - RB
    NT = 1 << TR
    assert launch[0] == NT
    blocks = np.arange(d.ntiles, dtype=np.int64)
    if d.xcd_remap:
        per = d.ntiles >> 3
        tile = (blocks & 7) * per + (blocks >> 3)
    else:
        tile = blocks
    base = np.zeros_like(tile)
    for b in range(d.nfree):
        base |= ((tile >> b) & 1) << P(d.free_w)[b]
    tid = np.arange(NT, dtype=np.int64)

    def dep_tid(pos):
        e = np.zeros(NT, dtype=np.int64)
        for b in range(TR):
            e |= ((tid >> b) & 1) << pos[b]
        return e

    def dep_reg(rho, pos):
        o = 0
        for q in range(RB):
            if (rho >> q) & 1:
                o |= 1 << pos[q]
        return o

    g = base[:, None] | dep_tid(P(d.ld_thr_w))[None, :]
    ld_idx = [g | dep_reg(rho, P(d.ld_reg_w)) for rho in range(R)]
    if check:
        allidx = np.concatenate([a.ravel() for a in ld_idx])
        assert np.unique(allidx).size == allidx.size == (1 << d.n), "loads are not a permutation"
    v = [src[i].astype(np.complex128) for i in ld_idx]
    if d.conj_in:
        v = [np.conj(a) for a in v]

    for gi in range(d.ngroups):
        G = d.grp[gi]
        e_thr = dep_tid(P(G.thr_w))
        if gi > 0:
            Gp = d.grp[gi - 1]
            e_prev = dep_tid(P(Gp.thr_w))
            lds = np.full((d.ntiles, 1 << T), np.nan + 0j)
            seen = np.zeros(1 << T, dtype=np.int64)
            for rho in range(R):
                a = _swizzle(e_prev | dep_reg(rho, P(Gp.reg_w)), c128)
                lds[:, a] = v[rho]
                np.add.at(seen, a, 1)
            if check:
                assert np.all(seen == 1), "LDS exchange does not cover the tile once"
            v = [lds[:, _swizzle(e_thr | dep_reg(rho, P(G.reg_w)), c128)] for rho in range(R)]
        # radix network with the constant twiddles of the register bits
        nst, jbase = G.nst, G.jbase
        for q in range(RB - 1, -1, -1):
            if q >= nst:
                continue
            for rho in range(R):
                if rho & (1 << q):
                    continue
                hi = rho | (1 << q)
                a, b = v[rho], v[hi]
                v[rho] = a + b
                J = (rho & ((1 << q) - 1)) << (4 - q)
                v[hi] = (a - b) * np.exp(-2j * np.pi * J / 32)
        # deferred phases of the thread's lower pass bits
        if jbase > 0 and nst > 0:
            u_thr = (e_thr >> d.pbase) & ((1 << jbase) - 1)
            MI1 = d.MI - 1
            f = []
            for q in range(RB):
                jl = jbase + q
                clear = max(0, jl - d.k) if d.aqft else 0
                x = np.zeros_like(u_thr) if clear >= jbase else (u_thr >> clear) << clear
                f.append(W[x << (MI1 - jl)] if q < nst else np.ones(NT, complex))
            for rho in range(1, R):
                F = np.ones(NT, complex)
                for q in range(RB):
                    if (rho >> q) & 1:
                        F = F * f[q]
                v[rho] = v[rho] * F[None, :]

    obase = _bitrev(base, d.n) if d.reverse else base
    g = obase[:, None] | dep_tid(P(d.st_thr_w))[None, :]
    nmask = (1 << d.n) - 1

    def omega(E):
        return tlo[E & ((1 << d.L) - 1)] * thi[E >> d.L]

    if d.ext_tw:
        vv = g & ((1 << d.lo) - 1)
        pt = (g >> d.lo) & ((1 << d.m) - 1)
        if not d.aqft:
            Et = (vv * _bitrev(pt, d.m)) << (d.n - d.lo - d.m)
        else:
            Et = np.zeros_like(g)
            for j in range(d.m):
                s = d.lo + j - d.k
                tv = vv if s <= 0 else (np.zeros_like(vv) if s >= d.lo else (vv >> s) << s)
                Et = (Et + np.where((pt >> j) & 1, tv << (d.n - 1 - d.lo - j), 0)) & nmask
        fq = []
        for q in range(RB):
            j = P(d.st_reg_w)[q] - d.lo
            assert 0 <= j < d.m, "a register bit of the store map is not a pass bit"
            s = d.lo + j - d.k
            tv = vv if (not d.aqft or s <= 0) else (np.zeros_like(vv) if s >= d.lo else (vv >> s) << s)
            fq.append(omega((tv << (d.n - 1 - d.lo - j)) & nmask))
        f0 = omega(Et) * d.scale
        for rho in range(R):
            F = f0.copy()
            for q in range(RB):
                if (rho >> q) & 1:
                    F = F * fq[q]
            v[rho] = v[rho] * F
    else:
        v = [x * d.scale for x in v]
    if d.conj_out:
        v = [np.conj(a) for a in v]
    out_idx, out_val = [], []
    for rho in range(R):
        idx = g | dep_reg(rho, P(d.st_reg_w))
        out_idx.append(idx.ravel())
        out_val.append(v[rho].ravel())
    out_idx = np.concatenate(out_idx)
    out_val = np.concatenate(out_val)
    if check:
        assert np.unique(out_idx).size == out_idx.size == (1 << d.n), "stores are not a permutation"
    return out_idx, out_val


def emulate(x, n, cutoff=-1, norm="unitary", dtype="c64", order="natural", config=None,
            inverse=False):
    layout = Q.layout_flags(dtype, order, "fused", inverse)
    c128 = bool(layout & Q.QFT_C128)
    info = Q.describe(n, cutoff, norm, dtype, order, "fused", config, inverse)
    tables = get_tables(n, cutoff, norm, layout, config)
    image, dt = get_table_image(n, cutoff, norm, layout, config)
    state = np.asarray(x, dtype=np.complex128).copy()
    ws = np.zeros_like(state)
    for p in range(info.num_passes):
        d, launch = get_pass(n, cutoff, norm, layout, config, p)
        check_group_table(d, launch, image, dt, tables[0])
        src = ws if launch[3] else state
        dst = ws if launch[4] else state
        idx, val = run_pass(d, launch, src, tables, c128)
        dst[idx] = val
    return state
