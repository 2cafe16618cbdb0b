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

namespace qft {

constexpr int kMaxTile = 15;   // max tile bits
constexpr int kMaxRadix = 5;   // max register bits (32 elements per thread)
constexpr int kMaxGroups = 15; // register groups per pass
constexpr int kMaxPasses = 8;

// Register/thread mapping of one group of stages.
// Element of thread `tid`, register `rho`:
//   e = deposit(tid, thr_pos) | deposit(rho, reg_pos).
struct GroupMap {
  uint8_t reg_pos[kMaxRadix];  // e-position of register bit q
  uint8_t thr_pos[kMaxTile];   // e-position of thread-id bit b
  int8_t jbase;                // local pass bit held by register bit 0
  int8_t nst;                  // stages (targets) applied in this group
};

struct PassDesc {
  // geometry
  uint8_t n;        // qubits of the transform
  uint8_t T;        // tile bits
  uint8_t r;        // register bits (R = 2^r)
  uint8_t m;        // pass bits
  uint8_t pbase;    // e-position of local pass bit 0
  uint8_t lo;       // target qubit of local pass bit 0
  uint8_t ngroups;  // register groups
  uint8_t reverse;  // 1: output index = rev_n(input index)
  uint8_t ext_tw;   // 1: apply the diagonal of controls below the pass
  uint8_t aqft;     // 1: cutoff < n - 1
  int8_t k;         // effective cutoff (max control-target distance kept)
  uint8_t nfree;    // non-tile index bits
  uint8_t MI;       // internal twiddle table: w_{2^MI}^y, y < 2^(MI-1)
  uint8_t L;        // split of the two-level w_N table
  uint8_t xcd_remap;// 1: XCD-aware tile order
  uint8_t pad_;
  uint32_t ntiles;
  uint8_t gpos[kMaxTile];     // global index bit of e-position q
  uint8_t free_pos[32];       // global positions of the non-tile bits, ascending
  // global (input / output) bit positions for the load group (group 0) and
  // the store group (last group)
  uint8_t ld_thr_g[kMaxTile];
  uint8_t ld_reg_g[kMaxRadix];
  uint8_t st_thr_g[kMaxTile];
  uint8_t st_reg_g[kMaxRadix];
  GroupMap grp[kMaxGroups];
  double scale;               // folded butterfly normalisation / output norm
  const void *tw_int;         // w_{2^MI}^y, y < 2^(MI-1)
  const void *tw_lo;          // w_N^x, x < 2^L
  const void *tw_hi;          // w_N^(x 2^L), x < 2^(n-L)
};

// Host-side description of one launch of the fused schedule.
struct PassLaunch {
  PassDesc d;
  int threads;        // workgroup size (2^(T - r))
  int lds_bytes;
  uint32_t grid;
  int in_ws;          // read from the workspace instead of the state
  int out_ws;         // write to the workspace instead of the state
};

}  // namespace qft
