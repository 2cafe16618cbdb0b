// Internal data structures shared by the host planner and the gfx950 kernels.
//
// A fused plan is a sequence of HBM passes.  Pass p applies the Hadamard
// butterflies and controlled phases of the target qubits [lo, lo + m) (in
// descending order, as in the circuit of Fig. 1) to every tile of the array.
// A tile is the set of 2^T indices obtained by varying T "tile bits": the m
// pass bits plus T - m spectator bits that only widen the contiguous memory
// runs a tile touches.  Inside a tile the pass is a batched 2^m-point
// decimation-in-frequency transform (butterflies + the controlled phases whose
// control lies in the pass), followed by one diagonal that collects every
// controlled phase whose control lies below the pass (those commute with the
// remaining butterflies of the pass, Sec. 2 gate fusion).
//
// Tile element index e (T bits): e-positions [0, pbase) are spectators,
// [pbase, pbase + m) are the pass bits (local bit j = target qubit lo + j).
// gpos[q] is the global index bit carried by e-position q.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#define __device__
#endif
#endif

namespace qft {

constexpr int kMaxTile = 15;   // max tile bits
constexpr int kMaxRadix = 5;   // max register bits (32 elements per thread)
constexpr int kMaxGroups = 15; // register groups per pass
constexpr int kMaxPasses = 8;

// Bit positions (0..31) are stored four per 32-bit word, so that device code
// reads them with scalar loads at wave-uniform indices and extracts bytes.
__host__ __device__ inline uint32_t pos_get(const uint32_t *w, int i) {
  return (w[i >> 2] >> ((i & 3) * 8)) & 0xffu;
}
inline void pos_set(uint32_t *w, int i, uint32_t v) {
  const int sh = (i & 3) * 8;
  w[i >> 2] = (w[i >> 2] & ~(0xffu << sh)) | ((v & 0xffu) << sh);
}

// Register/thread mapping of one group of stages.
// Element of thread `tid`, register `rho`:
//   e = deposit(tid, thr) | deposit(rho, reg).
struct GroupMap {
  uint32_t reg_w[2];  // e-position of register bit q (packed)
  uint32_t thr_w[4];  // e-position of thread-id bit b (packed)
  int32_t jbase;      // local pass bit held by register bit 0
  int32_t nst;        // stages (targets) applied in this group
};

struct PassDesc {
  // geometry
  int32_t n;        // qubits of the transform
  int32_t T;        // tile bits
  int32_t r;        // register bits (R = 2^r)
  int32_t m;        // pass bits
  int32_t pbase;    // e-position of local pass bit 0
  int32_t lo;       // target qubit of local pass bit 0
  int32_t ngroups;  // register groups
  int32_t reverse;  // 1: output index = rev_n(input index)
  int32_t ext_tw;   // 1: apply the diagonal of controls below the pass
  int32_t aqft;     // 1: cutoff < n - 1
  int32_t k;        // effective cutoff (max control-target distance kept)
  int32_t nfree;    // non-tile index bits
  int32_t MI;       // internal twiddle table: w_{2^MI}^y, y < 2^(MI-1)
  int32_t L;        // split of the two-level w_N table
  int32_t xcd_remap;// 1: XCD-aware tile order
  int32_t conj_in;  // 1: conjugate the loaded elements (first pass, inverse)
  int32_t conj_out; // 1: conjugate the stored elements (last pass, inverse)
  int32_t nt;       // 1: non-temporal (streaming) loads and stores
  int32_t lane_swap;// s > 0: three register groups, the last one taking pass
                    // bits 0..s-1 from lane bits 5..6-s of the middle group
                    // by cross-lane swaps (no LDS); 0 otherwise
  uint32_t ntiles;
  uint32_t gpos_w[4];   // global index bit of e-position q (packed)
  uint32_t free_w[8];   // global positions of the non-tile bits, ascending
  // global (input / output) bit positions for the load group (group 0) and
  // the store group (last group)
  uint32_t ld_thr_w[4];
  uint32_t ld_reg_w[2];
  uint32_t st_thr_w[4];
  uint32_t st_reg_w[2];
  GroupMap grp[kMaxGroups];
  double scale;               // folded butterfly normalisation / output norm
  const void *tw_int;         // w_{2^MI}^y, y < 2^(MI-1)
  const void *tw_lo;          // w_N^x, x < 2^L
  const void *tw_hi;          // w_N^(x 2^L), x < 2^(n-L)
  const void *gtab;           // per-thread factors of group 0, [q][tid]
                              // (entries of tw_int), or null
  const void *gtab1;          // the same for group 1 of a three-group pass
  double *norm_part;          // non-null: per-wave sums of |x|^2 of the
                              // loaded tile at [tile * parts_per_tile + w]
  const void *cmp_ref;        // last pass of a compare execute: reference
                              // output (same layout as the output), or null
  double *cmp_part;           // its per-wave comparison partials, kCmpSlots
                              // doubles each, at [tile * parts_per_tile + w]
};

// Slots of one comparison partial (FP64), in this order: sum |y - r|^2,
// sum |r|^2, sum |y|^2, Re and Im of sum conj(r) y, max |y - r|^2, max |r|^2
// and the lowest index where |r|^2 takes that maximum (as a double).
constexpr int kCmpSlots = 8;

// Partial sums of |x|^2 one workgroup of `threads` threads writes when a pass
// reduces the norm of its input: one per wave of 64, or one per thread when
// the workgroup is smaller than a wave.
inline int norm_parts_per_tile(int threads) { return threads >= 64 ? threads / 64 : threads; }

// Host-side description of one launch of the fused schedule.
struct PassLaunch {
  PassDesc d;
  int threads;        // workgroup size (2^(T - r))
  int lds_bytes;
  uint32_t grid;
  int in_ws;          // read from the workspace instead of the state
  int out_ws;         // write to the workspace instead of the state
};

// 0 for the generic pass kernel; 1 + 5 * ext + (nst - 1) for a pass with the
// two-group shape of the compile-time specialised kernel: radix 32, the
// first group full and carrying per-thread factors, the last group holding
// pass bit 0 with nst stages, every thread of the workgroup active.
inline int pass2_shape(const PassLaunch &L) {
  const PassDesc &d = L.d;
  const bool two = d.r == 5 && d.ngroups == 2 && d.grp[0].nst == d.r && d.grp[0].jbase > 0 &&
                   d.grp[1].jbase == 0 && d.grp[1].nst >= 1 && d.grp[1].nst <= d.r &&
                   L.threads == (1 << (d.T - d.r));
  return two ? 1 + (d.ext_tw ? 5 : 0) + (d.grp[1].nst - 1) : 0;
}

// 0, or 1 + 3 * ext + (s - 1) for a pass of 10 + s bits (s = 1..3) with the
// three-group shape of the compile-time kernel: radix 32, groups 0 and 1
// full and carrying per-thread factors, group 2 holding pass bits 0..s-1,
// which reach its registers by cross-lane swaps with lane bits 5, 4, 3.
inline int pass3_shape(const PassLaunch &L) {
  const PassDesc &d = L.d;
  const int s = d.lane_swap;
  const bool three = s >= 1 && s <= 3 && d.r == 5 && d.ngroups == 3 && d.m == 10 + s &&
                     d.grp[0].nst == 5 && d.grp[0].jbase == s + 5 && d.grp[1].nst == 5 &&
                     d.grp[1].jbase == s && d.grp[2].jbase == 0 && d.grp[2].nst == s &&
                     d.T - d.r >= 6 && L.threads == (1 << (d.T - d.r));
  return three ? 1 + (d.ext_tw ? 3 : 0) + (s - 1) : 0;
}

// 0, or nst (1..5) for a last pass with the two-group shape whose stores go
// through a third, exchange-only register group (the last pass of a
// bit-reversed-order plan, which holds the lowest output bits in registers
// for its final stages), with no below-pass diagonal and a full-tile LDS
// area of at most 64 KiB.
inline int pass2x_shape(const PassLaunch &L) {
  const PassDesc &d = L.d;
  const bool ok = d.r == 5 && d.ngroups == 3 && !d.ext_tw && d.grp[0].nst == d.r &&
                  d.grp[0].jbase > 0 && d.grp[1].jbase == 0 && d.grp[1].nst >= 1 &&
                  d.grp[1].nst <= d.r && d.grp[2].nst == 0 && d.lane_swap == 0 &&
                  L.threads == (1 << (d.T - d.r)) && L.lds_bytes <= 65536;
  return ok ? d.grp[1].nst : 0;
}

// Kernel of a pass: 0 generic, 1..10 the two-group kernel (pass2_shape),
// 11..16 the three-group kernel (10 + pass3_shape), 17..21 the two-group
// kernel with the store exchange (16 + pass2x_shape).
inline int pass_kernel_shape(const PassLaunch &L) {
  const int two = pass2_shape(L);
  if (two) return two;
  const int three = pass3_shape(L);
  if (three) return 10 + three;
  const int twox = pass2x_shape(L);
  return twox ? 16 + twox : 0;
}

// The lean (four-wave) form of the compile-time kernels runs every
// complex64 pass of 512 threads (2^14-element tiles) and every complex128
// one of 256 threads (2^13).
inline bool lean_form(const PassLaunch &L, bool c128) { return L.threads == (c128 ? 256 : 512); }

}  // namespace qft
