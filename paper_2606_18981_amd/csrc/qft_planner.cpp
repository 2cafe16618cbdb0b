// Host planner for the QFT->FFT schedule (pure C++, FP64 tables).
//
// Gate list (Fig. 1; cutoff semantics of Sec. 2 "Approximate QFT"):
//   for t = n-1 .. 0: H(t), then controlled-R_{d+1}(control t-d, target t)
//   for every distance d = 1 .. t with d <= k; finally swaps q_a <-> q_{n-1-a}.
//
// Fused schedule.  The targets are split, most significant first, into HBM
// passes of m consecutive qubits.  Within a pass every controlled phase whose
// control lies below the pass depends only on the target bit and on index
// bits no butterfly of the pass touches, so all of them commute to the end of
// the pass and collapse into one diagonal per element (Sec. 2 gate fusion:
// commuting diagonals collapse to one diagonal).  For the exact transform
// that diagonal is w_{2^{lo+m}}^{v rev_m(p)} (v = index bits below the pass,
// p = pass bits after the pass); for the AQFT each target's contribution
// keeps only the control bits within distance k.  The controlled phases with
// both qubits inside the pass become the twiddles of a 2^m-point
// decimation-in-frequency transform (Sec. 2 "From FFT to QFT": the diagonal
// T~ between two butterfly banks is the product of the two-level controlled
// phases).  The final swaps become the output addressing of the last pass
// (Sec. 3 step 2: the permutation is an index mapping, not a gate).
#include "qft_planner.h"

#include <math.h>
#include <string.h>

#include <algorithm>

namespace qft {

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct PassGeom {
  int lo = 0;
  int m = 0;
  std::vector<int> spec_g;  // global positions of the spectator bits
  bool reverse = false;
};

void put_cplx(std::vector<unsigned char> &buf, size_t off, size_t idx, bool c128,
              double re, double im) {
  if (c128) {
    double v[2] = {re, im};
    memcpy(buf.data() + off + idx * 16, v, 16);
  } else {
    float v[2] = {(float)re, (float)im};
    memcpy(buf.data() + off + idx * 8, v, 8);
  }
}

int check_config(const qft_config_t &c, std::string &err) {
  if (c.radix_log2 < 1 || c.radix_log2 > kMaxRadix) {
    err = "radix_log2 must be in [1, 5]";
    return QFT_ERR_INVALID;
  }
  if (c.tile_log2 < c.radix_log2 || c.tile_log2 > kMaxTile) {
    err = "tile_log2 must be in [radix_log2, 15]";
    return QFT_ERR_INVALID;
  }
  if (c.spec_log2 < 0 || c.spec_log2 >= c.tile_log2 || c.rev_spec_log2 < 0 ||
      c.rev_spec_log2 >= c.tile_log2) {
    err = "spec_log2 and rev_spec_log2 must be in [0, tile_log2)";
    return QFT_ERR_INVALID;
  }
  for (int i = 0; i < QFT_MAX_PASSES; ++i) {
    if (c.pass_tile_log2[i] < 0 || c.pass_tile_log2[i] > kMaxTile) {
      err = "pass_tile_log2 entries must be 0 (planner's choice) or at most 15";
      return QFT_ERR_INVALID;
    }
  }
  if ((1 << (c.tile_log2 - c.radix_log2)) > (c.radix_log2 >= 5 ? 512 : 1024)) {
    err = "too many threads per workgroup (2^(tile_log2 - radix_log2) must be <= 1024, "
          "or <= 512 for radix_log2 = 5)";
    return QFT_ERR_INVALID;
  }
  return QFT_OK;
}

// Register/thread maps of one pass.  See qft_internal.h for the meaning of
// the e-positions.  Groups apply the pass bits top-down, r at a time; the
// last (lowest) group may apply fewer and then also holds already-applied
// bits (or spectators) in its spare registers, which do not enter the
// twiddles of the lower targets.
void build_groups(PassLaunch &L, const PassGeom &g, int r, int n) {
  PassDesc &d = L.d;
  const int nspec = (int)g.spec_g.size();
  const int m = g.m;
  const int T = nspec + m;
  std::vector<int> gpos(T), outpos(T);
  for (int q = 0; q < T; ++q) {
    gpos[q] = q < nspec ? g.spec_g[q] : g.lo + (q - nspec);
    outpos[q] = g.reverse ? n - 1 - gpos[q] : gpos[q];
  }
  const int ng = (m + r - 1) / r;
  std::vector<GroupMap> groups;
  std::vector<std::vector<int>> thr_orders;
  for (int i = 0; i < ng; ++i) {
    const int top = m - i * r;
    const int bot = std::max(0, top - r);
    const int nst = top - bot;
    std::vector<int> regs;
    for (int q = 0; q < nst; ++q) regs.push_back(nspec + bot + q);
    if (nst < r) {
      // spare registers: applied pass bits above, then spectators
      std::vector<int> cand;
      for (int q = nspec + nst; q < nspec + m; ++q) cand.push_back(q);
      for (int q = 0; q < nspec; ++q) cand.push_back(q);
      for (int q : cand) {
        if ((int)regs.size() == r) break;
        if (std::find(regs.begin(), regs.end(), q) == regs.end()) regs.push_back(q);
      }
    }
    std::vector<int> thr;
    for (int q = 0; q < T; ++q)
      if (std::find(regs.begin(), regs.end(), q) == regs.end()) thr.push_back(q);
    if (i == 0) {
      std::stable_sort(thr.begin(), thr.end(), [&](int a, int b) { return gpos[a] < gpos[b]; });
    } else if (i == ng - 1) {
      std::stable_sort(thr.begin(), thr.end(), [&](int a, int b) { return outpos[a] < outpos[b]; });
    }
    GroupMap gm;
    memset(&gm, 0, sizeof(gm));
    for (int q = 0; q < r; ++q) pos_set(gm.reg_w, q, regs[q]);
    for (size_t b = 0; b < thr.size(); ++b) pos_set(gm.thr_w, (int)b, thr[b]);
    gm.jbase = bot;
    gm.nst = nst;
    groups.push_back(gm);
    thr_orders.push_back(thr);
  }
  // Three radix-32 groups whose last group holds s = 1..3 pass bits: the
  // middle group keeps pass bits 0..s-1 on lane bits 5, 4, 3 of its thread
  // map, so that the last group takes them into its low register bits by
  // cross-lane swaps with the middle group's register bits 0..s-1 instead of
  // an LDS exchange.  The remaining thread bits are ordered by output
  // address: after the swaps they are the store map, whose low lanes then
  // run along contiguous output memory.
  const int s_lane = m - 2 * r;
  if (r == 5 && ng == 3 && s_lane >= 1 && s_lane <= 3 && T - r >= 6 && nspec + s_lane <= 6) {
    std::vector<int> reg1(r), rest;
    for (int q = 0; q < r; ++q) reg1[q] = nspec + s_lane + q;
    for (int q = 0; q < T; ++q) {
      const bool low = q >= nspec && q < nspec + s_lane;
      if (!low && std::find(reg1.begin(), reg1.end(), q) == reg1.end()) rest.push_back(q);
    }
    std::stable_sort(rest.begin(), rest.end(), [&](int a, int b) { return outpos[a] < outpos[b]; });
    std::vector<int> thr1(T - r, -1);
    for (int q = 0; q < s_lane; ++q) thr1[5 - q] = nspec + q;
    size_t next = 0;
    for (int b = 0; b < T - r; ++b)
      if (thr1[b] < 0) thr1[b] = rest[next++];
    std::vector<int> reg2(r), thr2 = thr1;
    for (int q = 0; q < r; ++q) reg2[q] = q < s_lane ? nspec + q : reg1[q];
    for (int q = 0; q < s_lane; ++q) thr2[5 - q] = reg1[q];
    for (int q = 0; q < r; ++q) {
      pos_set(groups[1].reg_w, q, reg1[q]);
      pos_set(groups[2].reg_w, q, reg2[q]);
    }
    for (int b = 0; b < T - r; ++b) {
      pos_set(groups[1].thr_w, b, thr1[b]);
      pos_set(groups[2].thr_w, b, thr2[b]);
    }
    thr_orders[1] = thr1;
    thr_orders[2] = thr2;
    d.lane_swap = s_lane;
  }
  // A single group loads in input order; if the output order differs, add an
  // exchange-only group that stores in output order.
  if (ng == 1) {
    std::vector<int> thr = thr_orders[0];
    std::vector<int> by_out = thr;
    std::stable_sort(by_out.begin(), by_out.end(), [&](int a, int b) { return outpos[a] < outpos[b]; });
    if (by_out != thr) {
      GroupMap gm = groups[0];
      for (size_t b = 0; b < by_out.size(); ++b) pos_set(gm.thr_w, (int)b, by_out[b]);
      gm.nst = 0;
      gm.jbase = 0;
      groups.push_back(gm);
    }
  }
  // A multi-group pass whose last group holds the lowest output bits in
  // registers (the last pass of a bit-reversed-order plan: its pass bit 0 is
  // global bit 0) would have every lane of a store write to its own row of
  // memory.  An exchange-only group then puts the lowest output bits on the
  // lanes: registers on the r tile bits with the highest output positions,
  // threads on the rest in output order.
  auto lane_run = [&](const std::vector<int> &thr, const std::vector<int> &pos) {
    int k = 0;
    while (k < (int)thr.size() && pos[thr[k]] == k) ++k;  // global bits 0..k-1 on lanes
    return k;
  };
  if (ng >= 2) {
    std::vector<int> byout(T);
    for (int q = 0; q < T; ++q) byout[q] = q;
    std::stable_sort(byout.begin(), byout.end(),
                     [&](int a, int b) { return outpos[a] < outpos[b]; });
    const int run_st = lane_run(thr_orders.back(), outpos);
    // lanes of the exchange-only group's map: the tile's lowest output bits
    const int run_x = std::min(lane_run(byout, outpos), T - r);
    if (run_st < 3 && run_x >= run_st + 2) {
      GroupMap gm;
      memset(&gm, 0, sizeof(gm));
      for (int q = 0; q < r; ++q) pos_set(gm.reg_w, q, byout[T - r + q]);
      for (int b = 0; b < T - r; ++b) pos_set(gm.thr_w, b, byout[b]);
      gm.jbase = 0;
      gm.nst = 0;
      groups.push_back(gm);
      d.lane_swap = 0;  // the group maps then go through LDS only
    }
  }
  d.ngroups = (int)groups.size();
  for (size_t i = 0; i < groups.size(); ++i) d.grp[i] = groups[i];
  for (int q = 0; q < T; ++q) pos_set(d.gpos_w, q, gpos[q]);
  const GroupMap &g0 = groups.front();
  const GroupMap &gl = groups.back();
  for (int b = 0; b < T - r; ++b) {
    pos_set(d.ld_thr_w, b, gpos[pos_get(g0.thr_w, b)]);
    pos_set(d.st_thr_w, b, outpos[pos_get(gl.thr_w, b)]);
  }
  for (int q = 0; q < r; ++q) {
    pos_set(d.ld_reg_w, q, gpos[pos_get(g0.reg_w, q)]);
    pos_set(d.st_reg_w, q, outpos[pos_get(gl.reg_w, q)]);
  }
}

// log2 of the largest workgroup the kernel instance for (r, dtype) allows
// (its launch bounds keep the register tile of 2^r elements free of spills)
int max_thread_bits(int r, bool c128) {
  if (c128) return r >= 5 ? 8 : r >= 3 ? 9 : 10;
  return r >= 5 ? 9 : 10;
}

// Per-thread factors of a register group of a pass that a compile-time
// kernel runs (group 0 of the two-group shape, groups 0 and 1 of the
// three-group shape): entry [q][tid] is the internal-table entry
// w_{2^MI}^{x << (MI - 1 - jl)} that the group's factor for register bit q of
// thread tid reads (jl = jbase + q, x = the thread's lower pass bits with
// those below jl - k cleared for an AQFT).  Copying the table entry keeps the
// result bitwise the same as reading the table, while the kernel reads 64
// consecutive entries per wave instead of 64 scattered ones.  Returns the
// byte offset of the new table in the image.
size_t add_group_table(HostPlan &p, const PassLaunch &L, const GroupMap &G) {
  const size_t es = p.elem_bytes;
  const PassDesc &d = L.d;
  const int TR = d.T - d.r;
  const int threads = L.threads;
  const size_t off = p.tables.size();
  p.tables.resize(align_up(off + (size_t)d.r * threads * es, 256), 0);
  const int MI1 = d.MI - 1;
  for (int tid = 0; tid < threads; ++tid) {
    uint32_t e_thr = 0;
    for (int b = 0; b < TR; ++b) e_thr |= (uint32_t)((tid >> b) & 1) << pos_get(G.thr_w, b);
    const uint32_t u = (e_thr >> d.pbase) & ((1u << G.jbase) - 1u);
    for (int q = 0; q < d.r; ++q) {
      const size_t dst = off + ((size_t)q * threads + tid) * es;
      if (q >= G.nst) {
        put_cplx(p.tables, dst, 0, p.c128, 1.0, 0.0);
        continue;
      }
      const int jl = G.jbase + q;
      int clear = d.aqft ? jl - d.k : 0;
      clear = clear < 0 ? 0 : clear;
      const uint32_t x = clear >= G.jbase ? 0u : ((u >> clear) << clear);
      const size_t src = p.off_int + ((size_t)x << (MI1 - jl)) * es;
      memcpy(&p.tables[dst], &p.tables[src], es);
    }
  }
  return off;
}

void build_group_tables(HostPlan &p) {
  p.off_gtab.assign(p.passes.size(), 0);
  p.off_gtab1.assign(p.passes.size(), 0);
  for (size_t i = 0; i < p.passes.size(); ++i) {
    const PassLaunch &L = p.passes[i];
    if (pass2_shape(L) || pass2x_shape(L)) {
      p.off_gtab[i] = add_group_table(p, L, L.d.grp[0]);
    } else if (pass3_shape(L)) {
      p.off_gtab[i] = add_group_table(p, L, L.d.grp[0]);
      p.off_gtab1[i] = add_group_table(p, L, L.d.grp[1]);
    }
  }
}

int plan_fused(HostPlan &p, std::string &err) {
  const int n = p.n;
  const qft_config_t &c = p.cfg;
  int rc = check_config(c, err);
  if (rc) return rc;
  // Register radix: the controlled phases among a thread's register bits are
  // compile-time constants of the radix network, so for an AQFT every
  // register group must fit inside the cutoff distance (r <= k + 1).
  int r_cfg = c.radix_log2;
  if (p.keff < n - 1) r_cfg = std::min(r_cfg, p.keff + 1);
  const int T = std::min(c.tile_log2, r_cfg + max_thread_bits(r_cfg, p.c128));
  // A one-pass plan (the whole transform in one tile) is latency-bound:
  // take the fewest register groups, then the most threads.  Measured:
  // n = 11 complex128 9.9 us at radix 16 against 13.9 us at radix 32,
  // n = 12 complex64 10.6 against 13.9 us; n = 10 and 13 keep radix 32.
  if (p.auto_radix && n <= T && r_cfg == 5) {
    const int groups5 = (n + 4) / 5, groups4 = (n + 3) / 4;
    if (groups4 <= groups5 && n > 4) r_cfg = 4;
  }
  const int spec = std::min(c.spec_log2, T - 1);
  const int rspec = std::min(c.rev_spec_log2, T - 1);

  // Passes with qubits below them take one more tile bit in three-pass
  // plans of these sizes (see the tile rule below); the pass split and the
  // three-or-four-pass choice account for it.
  auto wide_sizes = [&](int P) {
    const bool size_ok = p.c128 ? (n >= 25 && n <= 30) : (n >= 28 && n <= 30);
    return size_ok && P == 3 && r_cfg == 5 &&
           T + 1 <= r_cfg + max_thread_bits(r_cfg, p.c128) && T + 1 <= kMaxTile;
  };

  // ---- pass partition --------------------------------------------------
  // widths[0] is the most significant pass; the last one holds qubit 0
  std::vector<int> widths;
  int nexplicit = 0, sum = 0;
  for (int i = 0; i < kMaxPasses; ++i) {
    if (c.pass_bits[i] < 0) {
      err = "pass_bits must be >= 0";
      return QFT_ERR_INVALID;
    }
    if (c.pass_bits[i] > 0) {
      if (nexplicit != i) {
        err = "pass_bits must be given from the first entry on, without gaps";
        return QFT_ERR_INVALID;
      }
      ++nexplicit;
      sum += c.pass_bits[i];
    }
  }
  if (nexplicit > 0) {
    if (sum != n) {
      err = "pass_bits must sum to n";
      return QFT_ERR_INVALID;
    }
    for (int i = 0; i < nexplicit; ++i) {
      if (c.pass_bits[i] > std::max(T, c.pass_tile_log2[i])) {
        err = "a pass cannot apply more qubits than the tile holds";
        return QFT_ERR_INVALID;
      }
      widths.push_back(c.pass_bits[i]);
    }
  } else if (n <= T) {
    widths.push_back(n);
  } else {
    const int b_eff = p.bitrev ? 0 : rspec;
    const int amax = T - b_eff;
    const int hmax = T - spec;
    int P = 2;
    while (amax + (P - 1) * hmax < n) ++P;
    if (P > kMaxPasses) {
      err = "too many passes for this tile configuration";
      return QFT_ERR_UNSUPPORTED;
    }
    if (P == 3 && P < kMaxPasses) {
      // A three-pass split whose first pass would read rows shorter than
      // 128 bytes takes a fourth pass instead: complex128 at n = 30 (64-byte
      // rows) measured 29.4 ms in three passes and 25.3 ms in four.
      const int rem = n - hmax;
      const int first = rem - std::max(std::min(amax, (rem + 1) / 2), rem - hmax);
      const int r0 = std::min(r_cfg, first);
      // see the first-pass and wide-tile rules below
      const int Tw = ((!p.c128 && T - first < 4) || wide_sizes(3)) ? T + 1 : T;
      const int Tp = std::min(Tw, r0 + max_thread_bits(r0, p.c128));
      const int spec0 = std::max(0, std::min(Tp - first, n - first));
      if ((p.elem_bytes << spec0) < 128) P = 4;
    }
    if (P <= 3) {
      // middle passes (rows close together in memory) as wide as the tile
      // allows; the first pass (rows 2^lo elements apart) and the last pass
      // (bit-reversed rows) share the rest evenly
      const int rem = n - (P - 2) * hmax;
      int a = std::max(std::min(amax, (rem + 1) / 2), rem - hmax);
      // A bit-reversing last pass of T - 4 bits (4 spectator bits) beats
      // the others, where the first pass still gets at least 6 bits and
      // rows of at least 256 bytes, or 128 bytes through the wider complex64
      // first-pass tile: complex64 n = 26 [7, 10, 9] 0.65 ms against
      // [8, 10, 8] 0.70 ms, n = 29 [10, 10, 9] 5.95 ms against [9, 10, 10]
      // 6.47 ms; complex128 n = 27 [9, 10, 8], whose first pass reads
      // 128-byte rows from a 2^12 tile, is 7 % slower than [8, 10, 9].
      if (P == 3 && !p.bitrev) {
        const int a4 = std::min(amax, T - 4), f4 = rem - a4;
        const bool wide = !p.c128 && T - f4 < 4;  // the first-pass rule below
        const int spec0 = std::min((wide ? T + 1 : T) - f4, n - f4);
        const size_t rows = p.elem_bytes << std::max(0, spec0);
        if (a4 != a && f4 >= 6 && f4 <= hmax && rows >= (wide ? 128u : 256u)) a = a4;
      }
      // A complex64 first pass that would hold T - 3 bits gives one bit to
      // an 11-bit middle pass of the three-group kernel, so that it keeps
      // T - 4 bits (n = 29: [9, 11, 9]).  With 2^13 tiles everywhere that
      // split took 5.82 ms against 6.00 for [10, 10, 9]; with the wider
      // high-pass tiles below all three measured 5.22 ms.  Not at n = 30:
      // [10, 11, 9] 11.23 ms against [10, 10, 10] 10.89 ms; nor at n = 28:
      // [8, 11, 9] 2.57 against [9, 10, 9] 2.45 ms.  (With 2^13 tiles the
      // 11-bit middle pass reads 32-byte rows, four tiles share each
      // 128-byte line, and L2 evicts it between them: 1.22x fetched, 1.32x
      // written.)
      int mid = hmax;
      if (P == 3 && !p.c128 && !p.bitrev && r_cfg == 5 && T - r_cfg >= 6 && rem - a == T - 3 &&
          n - (hmax + 1) - std::min(amax, T - 4) == T - 4 && hmax + 1 == 2 * r_cfg + 1 &&
          hmax + 1 <= T) {
        mid = hmax + 1;
        a = std::min(amax, T - 4);
      }
      widths.push_back(n - (P - 2) * mid - a);
      for (int i = 0; i < P - 2; ++i) widths.push_back(mid);
      widths.push_back(a);
    } else {
      // Four or more passes leave slack.  A bit-reversing last pass keeps
      // 4 spectator bits: narrower ones, with more and farther-apart row
      // groups, measured up to 3x slower at n = 31 (6 bits: 25.7 ms, 9 bits:
      // 6.9 ms).  The middle passes take the rounded-up share of the rest
      // and the first pass (rows farthest apart) what remains.
      int a = p.bitrev ? (n + P - 1) / P : std::min(amax, std::max(1, T - 4));
      if (n - a > (P - 1) * hmax) a = n - (P - 1) * hmax;
      const int rest = n - a;
      const int w = std::min(hmax, (rest + P - 2) / (P - 1));
      const int first = rest - (P - 2) * w;
      if (first >= 1) {
        widths.push_back(first);
        for (int i = 0; i < P - 2; ++i) widths.push_back(w);
      } else {  // tiny tiles: spread evenly
        const int q = rest / (P - 1), extra = rest % (P - 1);
        for (int i = 0; i < P - 1; ++i) widths.push_back(q + (i >= P - 1 - extra ? 1 : 0));
      }
      widths.push_back(a);
    }
  }
  std::vector<PassGeom> geo;
  {
    int top = n;
    const int P = (int)widths.size();
    // Complex64 passes below which other qubits lie take one more tile bit
    // in three-pass plans of 2^28 to 2^30 elements: 2^14-element tiles of
    // 512 threads, run by the four-wave form of the kernels (128 VGPRs, two
    // workgroups per CU), whose rows of 2^(tile - bits) contiguous elements
    // are twice as long.  n = 28: first pass 1.006 -> 0.856 ms (256-byte
    // rows), middle 0.800 -> 0.769 ms, 2.63 -> 2.45 ms in all; the
    // bit-reversing last pass keeps 2^13 (0.83 against 0.99 ms) unless its
    // rows would be shorter than 128 bytes (n = 30 [10, 10, 10]: 10.89 ms
    // with every pass at 2^14, 11.62 with the last at 2^13, 13.40 before).
    // n = 26, 27 and 31 measured 1-3 % slower with the wider tiles.
    // Complex128 likewise at 2^25..2^30 elements: 2^13-element tiles of 256
    // threads in the lean form (220 VGPRs, two waves per SIMD, split
    // exchange through 64 KiB of LDS: two workgroups per CU).  n = 28
    // 5.51 -> 4.78 ms (first pass 2.12 -> 1.64 ms with 256-byte rows),
    // n = 29 12.09 -> 9.66 ms, n = 30 23.6 ms in four passes -> 20.6 ms
    // in three, n = 26 and 27 3-6 % faster, n = 25 0.67 -> 0.63 ms (middle
    // pass 0.23 -> 0.20 ms with 128-byte rows); n = 24 within noise.
    const bool wide_high = wide_sizes(P);
    for (int i = 0; i < P; ++i) {
      PassGeom g;
      g.m = widths[i];
      g.lo = top - g.m;
      top = g.lo;
      int Tq = T;
      if (i < kMaxPasses && c.pass_tile_log2[i] > 0) {
        Tq = c.pass_tile_log2[i];
        if (Tq < g.m || Tq > kMaxTile) {
          err = "pass_tile_log2 must lie between the pass's qubits and 15";
          return QFT_ERR_INVALID;
        }
      } else if (wide_high &&
                 (i + 1 < P || (!p.bitrev && ((size_t)p.elem_bytes << (T - g.m)) < 128))) {
        // (a bit-reversing last pass with short rows; the last pass of a
        // bit-reversed-order plan stores whole tiles in input order)
        Tq = T + 1;
      } else if (i == 0 && !p.c128 && P >= 3 && T - g.m < 4) {
        // The first pass reads rows 2^lo elements apart; with fewer than 4
        // row bits (64-byte complex64 rows, at n = 30) one more tile bit is
        // worth the lower occupancy: measured 5.25 against 6.17 ms at n = 30.
        Tq = T + 1;
      }
      if (i + 1 < P) {
        // a high pass applies the diagonal of lower controls per register
        // group, which needs every register bit to be a pass bit (r <= m)
        const int r = std::min(r_cfg, g.m);
        const int Tp = std::min(Tq, r + max_thread_bits(r, p.c128));
        const int nspec = std::min(Tp - g.m, g.lo);
        for (int q = 0; q < nspec; ++q) g.spec_g.push_back(q);
      } else {
        g.reverse = !p.bitrev;
        const int Tp = std::min(Tq, std::min(r_cfg, Tq) + max_thread_bits(std::min(r_cfg, Tq), p.c128));
        const int nspec = std::min(std::max(Tp, g.m) - g.m, n - g.m);
        if (p.bitrev) {
          for (int q = 0; q < nspec; ++q) g.spec_g.push_back(g.m + q);
        } else {
          for (int q = 0; q < nspec; ++q) g.spec_g.push_back(n - nspec + q);
        }
      }
      geo.push_back(g);
    }
  }

  // ---- tables ------------------------------------------------------------
  int MI = 1;
  bool need_ext = false;
  for (const PassGeom &g : geo) {
    MI = std::max(MI, g.m);
    if (g.lo > 0) need_ext = true;
  }
  MI = std::max(MI, std::min(r_cfg, n));
  p.MI = MI;
  p.need_ext = need_ext;
  p.L = need_ext ? (n + 1) / 2 : 0;
  const size_t es = p.elem_bytes;
  const size_t n_int = (size_t)1 << (MI - 1);
  const size_t n_lo = need_ext ? ((size_t)1 << p.L) : 0;
  const size_t n_hi = need_ext ? ((size_t)1 << (n - p.L)) : 0;
  p.off_int = 0;
  p.off_lo = align_up(p.off_int + n_int * es, 256);
  p.off_hi = align_up(p.off_lo + n_lo * es, 256);
  p.tables.assign(align_up(p.off_hi + n_hi * es, 256), 0);
  p.end_hi = p.off_hi + n_hi * es;
  for (size_t y = 0; y < n_int; ++y) {
    double re, im;
    omega_pow2(MI, y, &re, &im);
    put_cplx(p.tables, p.off_int, y, p.c128, re, im);
  }
  for (size_t x = 0; x < n_lo; ++x) {
    double re, im;
    omega_pow2(n, x, &re, &im);
    put_cplx(p.tables, p.off_lo, x, p.c128, re, im);
  }
  for (size_t x = 0; x < n_hi; ++x) {
    double re, im;
    omega_pow2(n, (uint64_t)x << p.L, &re, &im);
    put_cplx(p.tables, p.off_hi, x, p.c128, re, im);
  }

  // ---- output scale: unit-norm butterflies folded per pass ---------------
  // total factor F = 2^{-n/2} * norm factor; passes other than the last get
  // the exact power of two 2^{-floor(m/2)}, the last gets the remainder.
  double F;
  if (p.norm == QFT_NORM_UNITARY) F = pow(2.0, -0.5 * n);
  else if (p.norm == QFT_NORM_NONE) F = 1.0;
  else F = pow(2.0, -1.0 * n);
  std::vector<double> scales(geo.size());
  double used = 1.0;
  for (size_t i = 0; i + 1 < geo.size(); ++i) {
    scales[i] = ldexp(1.0, -(geo[i].m / 2));
    used *= scales[i];
  }
  scales.back() = F / used;

  // ---- launches ------------------------------------------------------------
  const bool natural_multi = !p.bitrev && geo.size() > 1;
  p.ws_bytes = natural_multi ? p.state_bytes : 0;
  for (size_t i = 0; i < geo.size(); ++i) {
    const PassGeom &g = geo[i];
    PassLaunch L;
    memset(&L, 0, sizeof(L));
    PassDesc &d = L.d;
    const int Te = (int)g.spec_g.size() + g.m;
    int r = std::min(r_cfg, Te);
    if (g.lo > 0) r = std::min(r, g.m);
    d.n = n;
    d.T = Te;
    d.r = r;
    d.m = g.m;
    d.pbase = (int)g.spec_g.size();
    d.lo = g.lo;
    d.reverse = g.reverse ? 1 : 0;
    // inverse: conj(F conj(x)) runs the conjugate-phase circuit with the
    // forward tables; the conjugations ride on the first load and last store
    d.conj_in = (p.inverse && i == 0) ? 1 : 0;
    d.conj_out = (p.inverse && i + 1 == geo.size()) ? 1 : 0;
    d.ext_tw = g.lo > 0 ? 1 : 0;
    d.aqft = p.keff < n - 1 ? 1 : 0;
    d.k = p.keff;
    d.MI = MI;
    d.L = p.L;
    build_groups(L, g, r, n);
    // Non-tile bits, in the order in which the tile number fills them.
    // Workgroups with consecutive numbers run at the same time, so the low
    // tile-number bits go to the non-tile bits nearest the bottom of the
    // address that the pass writes: ascending input bits for a pass that
    // writes in place, descending for the bit-reversing pass (input bit b is
    // output bit n-1-b).  Concurrent workgroups then write neighbouring
    // memory.
    std::vector<int> in_tile(n, 0);
    for (int q = 0; q < Te; ++q) in_tile[pos_get(d.gpos_w, q)] = 1;
    int nf = 0;
    for (int j = 0; j < n; ++j) {
      const int b = g.reverse ? n - 1 - j : j;
      if (!in_tile[b]) pos_set(d.free_w, nf++, b);
    }
    d.nfree = nf;
    d.ntiles = 1u << nf;
    d.scale = scales[i];
    L.threads = 1 << (Te - r);
    L.lds_bytes = d.ngroups > 1 ? (int)(((size_t)1 << Te) * es) : 0;
    // the complex64 two-group kernel exchanges real and imaginary parts in
    // turn through half the tile's LDS (three workgroups per CU at 2^13)
    // and so does the lean complex128 form (2^13-element tiles, 256 threads)
    if ((!p.c128 || L.threads == 256) && (pass2_shape(L) || pass3_shape(L))) L.lds_bytes /= 2;
    L.grid = d.ntiles;
    // Streaming loads and stores pay off where a tile reads whole 128-byte
    // lines: where it reads half lines, the neighbouring tile (run at the
    // same time on the same XCD) reads the other half from L2.  They are
    // used only when the state is at least as large as the 256 MB Infinity
    // Cache (measured: 2^24 complex64 passes are faster cached, 2^25 and
    // 2^24 complex128 ones faster streaming).
    {
      int run = 0;  // low index bits held by the tile: contiguous run 2^run
      while (run < n && in_tile[run]) ++run;
      const bool lines = (es << run) >= 128;
      const bool big = p.state_bytes >= ((size_t)256 << 20);
      // (only the compile-time kernels have a streaming form)
      const bool want = (c.nontemporal == 2 && lines) || (c.nontemporal == 0 && lines && big);
      d.nt = want && (pass2_shape(L) || pass3_shape(L)) ? 1 : 0;
    }
    d.xcd_remap = (L.grid >= 8 && L.grid % 8 == 0) ? 1 : 0;
    if (natural_multi) {
      L.in_ws = i == 0 ? 0 : 1;
      L.out_ws = i + 1 == geo.size() ? 0 : 1;
    }
    p.passes.push_back(L);
  }
  build_group_tables(p);
  return QFT_OK;
}

void plan_gates(HostPlan &p) {
  const int n = p.n;
  for (int t = n - 1; t >= 0; --t) {
    Gate h{0, t, 0, 0, 0.0, 0.0};
    p.gates.push_back(h);
    for (int d = 1; d <= t; ++d) {
      if (d > p.keff) break;
      Gate g{1, t - d, t, d + 1, 0.0, 0.0};
      omega_pow2(d + 1, 1, &g.re, &g.im);  // R_{d+1}: exp(-2 pi i / 2^{d+1})
      if (p.inverse) g.im = -g.im;         // R_{d+1}^* for the inverse
      p.gates.push_back(g);
    }
  }
  if (!p.bitrev)
    for (int a = 0; a < n / 2; ++a) p.gates.push_back(Gate{2, a, n - 1 - a, 0, 0.0, 0.0});
  if (p.norm == QFT_NORM_UNITARY) p.gate_norm = 1.0;
  else if (p.norm == QFT_NORM_NONE) p.gate_norm = pow(2.0, 0.5 * n);
  else p.gate_norm = pow(2.0, -0.5 * n);
}

}  // namespace

qft_config_t default_config(bool c128) {
  qft_config_t c;
  memset(&c, 0, sizeof(c));
  // fastest measured at 2^27-2^28 elements (64 KiB tiles, radix 32)
  if (c128) {
    c.tile_log2 = 12;
    c.radix_log2 = 5;
    c.spec_log2 = 2;
    c.rev_spec_log2 = 2;
  } else {
    c.tile_log2 = 13;
    c.radix_log2 = 5;
    c.spec_log2 = 3;
    c.rev_spec_log2 = 3;
  }
  return c;
}

void omega_pow2(int logN, uint64_t m, double *re, double *im) {
  if (logN <= 0) {
    *re = 1.0;
    *im = 0.0;
    return;
  }
  const uint64_t N = 1ULL << logN;
  m &= N - 1;
  // m = q N/4 + r with 0 <= r < N/4; w_N^m = (-i)^q w_N^r
  int q;
  uint64_t r;
  if (logN >= 2) {
    q = (int)(m >> (logN - 2));
    r = m & ((N >> 2) - 1);
  } else {
    q = (int)(2 * m);  // N = 2: w_2 = -1 = (-i)^2
    r = 0;
  }
  const long double twopi = 6.283185307179586476925286766559L;
  long double cs, sn;  // cos and sin of 2 pi r / N, first octant reduced
  if (logN >= 3 && r > (N >> 3)) {
    const long double a = twopi * (long double)((N >> 2) - r) / (long double)N;
    cs = sinl(a);
    sn = cosl(a);
  } else {
    const long double a = twopi * (long double)r / (long double)N;
    cs = cosl(a);
    sn = sinl(a);
  }
  long double zr = cs, zi = -sn;
  for (int i = 0; i < q; ++i) {  // multiply by -i
    const long double t = zr;
    zr = zi;
    zi = -t;
  }
  *re = (double)zr;
  *im = (double)zi;
}

size_t HostPlan::hbm_bytes() const {
  if (schedule == Schedule::Fused) return 2 * state_bytes * passes.size();
  size_t b = 0;
  for (const Gate &g : gates) {
    if (g.kind == 0) b += 2 * state_bytes;      // every pair read and written
    else if (g.kind == 1) b += state_bytes / 2; // quarter of the amplitudes
    else b += state_bytes;                      // half of the amplitudes move
  }
  if (gate_norm != 1.0) b += 2 * state_bytes;
  return b;
}

int build_host_plan(int n, int cutoff, int norm, int layout, const qft_config_t *cfg,
                    HostPlan &p, std::string &err) {
  if (n < 1 || n > QFT_MAX_QUBITS) {
    err = "n must be in [1, " + std::to_string(QFT_MAX_QUBITS) + "]";
    return QFT_ERR_INVALID;
  }
  if (norm != QFT_NORM_UNITARY && norm != QFT_NORM_NONE && norm != QFT_NORM_INV_N) {
    err = "norm must be QFT_NORM_UNITARY, QFT_NORM_NONE or QFT_NORM_INV_N";
    return QFT_ERR_INVALID;
  }
  if (layout & ~(0x1F | QFT_PLAN_TUNED)) {
    err = "unknown layout flag bits";
    return QFT_ERR_INVALID;
  }
  p = HostPlan();
  p.n = n;
  p.keff = (cutoff < 0 || cutoff >= n - 1) ? n - 1 : cutoff;
  p.norm = norm;
  p.layout = layout;
  p.c128 = (layout & QFT_C128) != 0;
  p.bitrev = (layout & QFT_ORDER_BITREV) != 0;
  p.inverse = (layout & QFT_INVERSE) != 0;
  p.schedule = (layout & QFT_SCHEDULE_GATES) ? Schedule::Gates : Schedule::Fused;
  p.elem_bytes = p.c128 ? 16 : 8;
  p.state_bytes = p.elem_bytes << n;
  p.gates_h = n;
  p.gates_cr = (long long)p.keff * n - (long long)p.keff * (p.keff + 1) / 2;
  p.gates_swap = n / 2;
  qft_config_t def = default_config(p.c128);
  qft_config_t c = def;
  if (cfg) {
    if (cfg->tile_log2) c.tile_log2 = cfg->tile_log2;
    if (cfg->radix_log2) c.radix_log2 = cfg->radix_log2;
    if (cfg->spec_log2) c.spec_log2 = cfg->spec_log2 < 0 ? 0 : cfg->spec_log2;
    if (cfg->rev_spec_log2) c.rev_spec_log2 = cfg->rev_spec_log2 < 0 ? 0 : cfg->rev_spec_log2;
    c.nontemporal = cfg->nontemporal;
    c.spec_log2 = std::min(c.spec_log2, c.tile_log2 - 1);
    c.rev_spec_log2 = std::min(c.rev_spec_log2, c.tile_log2 - 1);
    for (int i = 0; i < QFT_MAX_PASSES; ++i) c.pass_bits[i] = cfg->pass_bits[i];
    for (int i = 0; i < QFT_MAX_PASSES; ++i) c.pass_tile_log2[i] = cfg->pass_tile_log2[i];
  }
  p.cfg = c;
  p.auto_radix = !cfg || cfg->radix_log2 == 0;
  if (p.schedule == Schedule::Gates) {
    plan_gates(p);
    return QFT_OK;
  }
  return plan_fused(p, err);
}

void describe_plan(const HostPlan &p, qft_plan_info_t *o) {
  memset(o, 0, sizeof(*o));
  o->n = p.n;
  o->cutoff = p.keff;
  o->norm = p.norm;
  o->layout = p.layout;
  o->config = p.cfg;
  o->gates_h = p.gates_h;
  o->gates_cr = p.gates_cr;
  o->gates_swap = p.bitrev ? 0 : p.gates_swap;
  o->state_bytes = p.state_bytes;
  o->workspace_bytes = p.ws_bytes;
  o->table_bytes = p.tables.size();
  o->hbm_bytes = p.hbm_bytes();
  if (p.schedule == Schedule::Fused) {
    o->num_passes = (int)p.passes.size();
    for (size_t i = 0; i < p.passes.size() && i < QFT_MAX_PASSES; ++i) {
      const PassDesc &d = p.passes[i].d;
      o->pass_lo[i] = d.lo;
      o->pass_bits[i] = d.m;
      o->pass_spec[i] = d.pbase;
      o->pass_reverse[i] = d.reverse;
      o->pass_kernel[i] = pass_kernel_shape(p.passes[i]);
      o->pass_streaming[i] = d.nt;
    }
  } else {
    o->num_passes = (int)p.gates.size() + (p.gate_norm != 1.0 ? 1 : 0);
  }
}

}  // namespace qft
