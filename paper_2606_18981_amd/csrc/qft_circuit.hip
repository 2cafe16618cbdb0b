// General fused-circuit execution: runs of one- and two-qubit gates applied
// to tiles of the state held in LDS, one HBM pass per run; see
// include/qft_circuit.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <string>
#include <vector>

#include "../../include/qft_circuit.h"
#include "qft_internal.h"
#include "qft_kernels.h"

namespace qft {
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
void clear_error();
}  // namespace qft

using namespace qft;

namespace {

constexpr int kCircThreads = 256;
constexpr int kMaxTileC64 = 13;   // 2^13 complex64 = 64 KiB of LDS (plus padding)
constexpr int kMaxTileC128 = 12;  // 2^12 complex128 = 64 KiB of LDS (plus padding)
constexpr int kLowBits = 6;       // tile positions [0, 6) index the low tables
constexpr int32_t kNoControl = 0x7fffffff;
constexpr int kChunk = 8;  // elements a thread scales per read of a diagonal record
constexpr int kLoadBatch = 16;  // tile loads a thread has in flight at once

// Per element type: high tile bits (T - 6), stage size (tile positions whose
// 2^K elements a thread holds in registers) and diagonal-run tables per stage.
template <typename Real>
struct Shape {
  static constexpr int kHighBits = (sizeof(Real) == 8 ? kMaxTileC128 : kMaxTileC64) - kLowBits;
  static constexpr int kStageBits = sizeof(Real) == 8 ? 4 : 5;
  static constexpr int kSlots = sizeof(Real) == 8 ? 4 : 5;
};

template <typename Real>
struct alignas(2 * sizeof(Real)) c2 {
  Real x, y;
};

enum GateKind : int32_t { kOne = 0, kControlled = 1, kSwap = 2 };

struct GateRec {
  int32_t kind;
  int32_t a, b;    // one-qubit: target a; controlled: control a, target b; swap: a, b
  double u[8];     // row-major 2x2, (re, im) pairs
};

// What a pass does, in order.  A qubit operand is encoded as its tile
// position p >= 0, or as -1 - g for a global bit g outside the tile (whose
// value is the same for every element of a tile).
//  - kOpStage: header of a stage, followed by its kOpPair operations.  The
//    stage's targets are at most kStageBits tile positions; every thread
//    holds the 2^K elements of a sub-cube over them in registers and applies
//    all the stage's gates (and their diagonal runs) there.
//  - kOpPair: a 2x2 matrix on the stage position with index `a`, optionally
//    controlled, then the diagonal run that follows it in the circuit.
//  - kOpDiag: a diagonal run with no non-diagonal gate before it in the pass.
// Swaps move no data in the pass: they relabel tile positions, operands are
// LDS (physical) positions, and the store applies the final relabelling.
// A diagonal run (consecutive diagonal gates, which commute) has its records
// split over a low table (low tile positions, global bits and at most one
// high position hx), a high table (high positions and global bits) and a
// list evaluated per element (gates pairing a low position with a high
// position other than hx).  The tables are built per tile.
enum OpKind : int32_t { kOpPair = 0, kOpDiag = 2, kOpStage = 3 };

// Pair-operation flags.  kRealMatrix: the 2x2 matrix is real (H, X, Z,
// rotations about Y, ...), two real multiply-adds per output component
// instead of four.  kAnchoredRun: every record of the run that follows the
// pair involves the pair's target and scales only amplitudes where all its
// qubits are 1 (controlled phases onto the target, phase gates on it), so the
// run's factor is 1 wherever the target bit is 0 and those elements are
// skipped.
enum OpFlags : int32_t { kRealMatrix = 1, kAnchoredRun = 2 };

template <typename Real>
struct DevOp {
  int32_t kind;
  int32_t a;       // pair: stage index of the target; swap: tile position;
                   // stage: number of pair operations that follow
  int32_t b;       // pair: encoded control or kNoControl; swap: tile position;
                   // stage: number of positions K
  int32_t r0;      // run: first record; stage: positions, 4 bits each, ascending
  int32_t nlo, nhi, ncross;  // run: records in the low table, high table, per element
                             // (stage: nlo = number of runs)
  int32_t hx;      // run: high tile position that extends the low table, or -1
  int32_t slot;    // pair: table slot of its run
  int32_t flags;   // pair: kRealMatrix, kAnchoredRun
  int32_t apos;    // pair with kAnchoredRun: tile position of its target
  int32_t pad;
  c2<Real> u[4];   // pair: row-major 2x2
};

// A diagonal gate on qubits (q1, q0): the amplitude is scaled by
// D[2 bit(q1) + bit(q0)] (q1 == q0 for a one-qubit diagonal).
template <typename Real>
struct DevDiag {
  int32_t q1, q0;
  int32_t pad[2];
  c2<Real> D[4];
};

struct CircPass {
  int32_t n, T, TL, nfree;
  int32_t nops;
  int32_t has_perm;     // the pass ends with swaps, folded into the store
  uint32_t perm_w[4];   // store: bit q of a tile element comes from position perm[q]
  uint32_t gpos_w[4];   // global bit of tile position q (packed 4 per word)
  uint32_t free_w[8];   // global bits of the non-tile positions, ascending
  uint32_t ntiles;
  int32_t xcd_remap;
  const void *ops;      // DevOp<Real>[nops]
  const void *recs;     // DevDiag<Real>[] of this pass
};

__device__ __forceinline__ uint32_t insert_zero(uint32_t x, int pos) {
  const uint32_t low = (1u << pos) - 1u;
  return ((x & ~low) << 1) | (x & low);
}

// LDS slot of tile element e: one pad element per 32 spreads the banks of
// sweeps whose lanes step over a gap of tile positions.
__device__ __forceinline__ uint32_t lidx(uint32_t e) { return e + (e >> 5); }

template <typename Real>
__device__ __forceinline__ c2<Real> cmul2(c2<Real> a, c2<Real> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename Real>
__device__ __forceinline__ c2<Real> cadd2(c2<Real> a, c2<Real> b) {
  return {a.x + b.x, a.y + b.y};
}

__device__ __forceinline__ uint32_t qbit(int32_t q, uint32_t e, uint64_t base) {
  return q >= 0 ? (e >> q) & 1u : (uint32_t)(base >> (-1 - q)) & 1u;
}

template <typename Real>
__device__ __forceinline__ c2<Real> diag_factor(const DevDiag<Real> &r, uint32_t e,
                                                uint64_t base) {
  const uint32_t b1 = qbit(r.q1, e, base), b0 = qbit(r.q0, e, base);
  const c2<Real> lo = b0 ? r.D[1] : r.D[0];
  const c2<Real> hi = b0 ? r.D[3] : r.D[2];
  return b1 ? hi : lo;
}

template <typename Real>
struct RunTables {
  c2<Real> lo[2 << kLowBits];
  c2<Real> hi[1 << Shape<Real>::kHighBits];
};

// Product of the factors of records [r0, r1) at tile element e.  The
// records are read four at a time before any is used, so that their scalar
// loads are in flight together rather than one round trip per record.
template <typename Real>
__device__ __forceinline__ c2<Real> record_product(const DevDiag<Real> *__restrict__ recs, int r0,
                                                   int r1, uint32_t e, uint64_t base) {
  c2<Real> f{(Real)1, (Real)0};
  int r = r0;
  for (; r + 4 <= r1; r += 4) {
    DevDiag<Real> rr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) rr[k] = recs[r + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) f = cmul2(f, diag_factor(rr[k], e, base));
  }
  for (; r < r1; ++r) f = cmul2(f, diag_factor(recs[r], e, base));
  return f;
}

// The factor tables of a diagonal run for this tile: thread j < 2^(TL+1)
// computes low entry j, thread 128 + j high entry j.
template <typename Real>
__device__ __forceinline__ void build_tables(const DevOp<Real> &op,
                                             const DevDiag<Real> *__restrict__ recs,
                                             RunTables<Real> &tb, int TL, int TH, uint64_t base,
                                             uint32_t tid) {
  using C = c2<Real>;
  const uint32_t mlo = (1u << TL) - 1u;
  const int hx = op.hx;
  // an anchored run's factor is 1 wherever its anchor bit is 0
  const int ap = (op.kind == kOpPair && (op.flags & kAnchoredRun)) ? op.apos : -1;
  if (tid < 128u) {
    if (tid <= mlo || (hx >= 0 && tid <= 2u * mlo + 1u)) {
      const uint32_t e = (tid & mlo) | (hx >= 0 ? ((tid >> TL) & 1u) << hx : 0u);
      C f{(Real)1, (Real)0};
      const bool skip = ap >= 0 && (ap < TL || ap == hx) && ((e >> ap) & 1u) == 0u;
      if (!skip) f = record_product<Real>(recs, op.r0, op.r0 + op.nlo, e, base);
      tb.lo[tid] = f;
    }
  } else if (tid - 128u < (1u << TH)) {
    const uint32_t j = tid - 128u;
    C f{(Real)1, (Real)0};
    const bool skip = ap >= TL && ((j >> (ap - TL)) & 1u) == 0u;
    if (!skip) f = record_product<Real>(recs, op.r0 + op.nlo, op.r0 + op.nlo + op.nhi, j << TL, base);
    tb.hi[j] = f;
  }
}

// Table part of a run's factor for tile element e.
template <typename Real>
__device__ __forceinline__ c2<Real> table_factor(const RunTables<Real> &tb, uint32_t e, int TL,
                                                 int hx) {
  const uint32_t mlo = (1u << TL) - 1u;
  const uint32_t xb = hx >= 0 ? ((e >> hx) & 1u) << TL : 0u;
  return cmul2(tb.lo[(e & mlo) | xb], tb.hi[e >> TL]);
}

// Matrix u on the register pairs (c, c + 2^J) of a sub-cube whose corner c
// is tile element eb | off[c]; where the control bit of a pair is clear it
// is left alone.
template <typename Real, int K, int J>
__device__ __forceinline__ void stage_pair(c2<Real> (&v)[1 << K], uint32_t eb,
                                           const uint32_t (&off)[1 << K], int cq, uint64_t base,
                                           c2<Real> u0, c2<Real> u1, c2<Real> u2, c2<Real> u3) {
  using C = c2<Real>;
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    if (c & (1 << J)) continue;
    const int c1 = c | (1 << J);
    const bool take = cq == kNoControl || qbit(cq, eb | off[c], base);
    const C a = v[c], b = v[c1];
    const C na = cadd2(cmul2(u0, a), cmul2(u1, b));
    const C nb = cadd2(cmul2(u2, a), cmul2(u3, b));
    v[c] = take ? na : a;
    v[c1] = take ? nb : b;
  }
}

// The same for a real matrix (u0..u3 the real parts).
template <typename Real, int K, int J>
__device__ __forceinline__ void stage_pair_real(c2<Real> (&v)[1 << K], uint32_t eb,
                                                const uint32_t (&off)[1 << K], int cq,
                                                uint64_t base, Real u0, Real u1, Real u2,
                                                Real u3) {
  using C = c2<Real>;
#pragma unroll
  for (int c = 0; c < (1 << K); ++c) {
    if (c & (1 << J)) continue;
    const int c1 = c | (1 << J);
    const bool take = cq == kNoControl || qbit(cq, eb | off[c], base);
    const C a = v[c], b = v[c1];
    const C na{u0 * a.x + u1 * b.x, u0 * a.y + u1 * b.y};
    const C nb{u2 * a.x + u3 * b.x, u2 * a.y + u3 * b.y};
    v[c] = take ? na : a;
    v[c1] = take ? nb : b;
  }
}

// One stage over K tile positions (packed ascending in `packed`): each
// thread takes sub-cubes s = tid + 256 i, loads their 2^K elements from LDS,
// applies the stage's operations in order and stores them back.
template <typename Real, int K>
__device__ __forceinline__ void stage_sweep(c2<Real> *lds, const DevOp<Real> *sops, int nsops,
                                            uint32_t packed, const RunTables<Real> *tabs,
                                            const DevDiag<Real> *recs, uint64_t base, int TL,
                                            uint32_t TE, uint32_t tid) {
  using C = c2<Real>;
  constexpr int R = 1 << K;
  int pos[K];
#pragma unroll
  for (int j = 0; j < K; ++j) pos[j] = (int)((packed >> (4 * j)) & 15u);
  uint32_t off[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) o |= (uint32_t)((c >> j) & 1) << pos[j];
    off[c] = o;
  }
  for (uint32_t s = tid; s < (TE >> K); s += kCircThreads) {
    uint32_t eb = s;
#pragma unroll
    for (int j = 0; j < K; ++j) eb = insert_zero(eb, pos[j]);
    C v[R];
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = lds[lidx(eb | off[c])];
    for (int oi = 0; oi < nsops; ++oi) {
      const DevOp<Real> &op = sops[oi];
      const C u0 = op.u[0], u1 = op.u[1], u2 = op.u[2], u3 = op.u[3];
      const int cq = op.b;
      const int J = op.a;
      if (op.flags & kRealMatrix) {
        switch (J) {
          case 0: stage_pair_real<Real, K, 0>(v, eb, off, cq, base, u0.x, u1.x, u2.x, u3.x); break;
          case 1: if constexpr (K > 1) stage_pair_real<Real, K, 1>(v, eb, off, cq, base, u0.x, u1.x, u2.x, u3.x); break;
          case 2: if constexpr (K > 2) stage_pair_real<Real, K, 2>(v, eb, off, cq, base, u0.x, u1.x, u2.x, u3.x); break;
          case 3: if constexpr (K > 3) stage_pair_real<Real, K, 3>(v, eb, off, cq, base, u0.x, u1.x, u2.x, u3.x); break;
          case 4: if constexpr (K > 4) stage_pair_real<Real, K, 4>(v, eb, off, cq, base, u0.x, u1.x, u2.x, u3.x); break;
          default: break;
        }
      } else {
        switch (J) {
          case 0: stage_pair<Real, K, 0>(v, eb, off, cq, base, u0, u1, u2, u3); break;
          case 1: if constexpr (K > 1) stage_pair<Real, K, 1>(v, eb, off, cq, base, u0, u1, u2, u3); break;
          case 2: if constexpr (K > 2) stage_pair<Real, K, 2>(v, eb, off, cq, base, u0, u1, u2, u3); break;
          case 3: if constexpr (K > 3) stage_pair<Real, K, 3>(v, eb, off, cq, base, u0, u1, u2, u3); break;
          case 4: if constexpr (K > 4) stage_pair<Real, K, 4>(v, eb, off, cq, base, u0, u1, u2, u3); break;
          default: break;
        }
      }
      if (op.nlo + op.nhi + op.ncross > 0) {
        const RunTables<Real> &tb = tabs[op.slot];
        const int hx = op.hx;
        // an anchored run leaves the elements whose target bit is 0 alone
        const uint32_t keep = (op.flags & kAnchoredRun) ? 1u << J : 0u;
#pragma unroll
        for (int c = 0; c < R; ++c)
          if (keep == 0u || (c & keep))
            v[c] = cmul2(table_factor<Real>(tb, eb | off[c], TL, hx), v[c]);
        const int rc0 = op.r0 + op.nlo + op.nhi, rc1 = rc0 + op.ncross;
        for (int r = rc0; r < rc1; ++r) {
          const DevDiag<Real> rec = recs[r];
#pragma unroll
          for (int c = 0; c < R; ++c)
            if (keep == 0u || (c & keep)) v[c] = cmul2(diag_factor(rec, eb | off[c], base), v[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) lds[lidx(eb | off[c])] = v[c];
  }
}

// One pass: load the tile into LDS (element e = sum over tile positions q of
// bit q of e at global bit gpos[q], plus the tile's free bits), apply the
// pass's operations in order (stages in registers, lone diagonal runs as LDS
// sweeps), one barrier after each, and store the tile through the pass's
// relabelling of tile positions (its swaps).
// (Two waves per SIMD: the LDS of two workgroups fits a CU, and the
// register budget of two waves is what the stage code needs.)
// FULL: every stage has Shape::kStageBits positions (tiles of at least that
// many bits); otherwise stages of 1..kStageBits positions.
// The operations and diagonal records come in as their own read-only,
// non-aliasing arguments: the compiler then reads them (wave-uniform) with
// scalar loads instead of vector loads through the vector cache.
template <typename Real, bool FULL>
__global__ void __launch_bounds__(kCircThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_circuit_pass(const CircPass d, c2<Real> *__restrict__ psi,
               const DevOp<Real> *__restrict__ ops, const DevDiag<Real> *__restrict__ recs) {
  using C = c2<Real>;
  using S = Shape<Real>;
  extern __shared__ __align__(16) unsigned char circ_smem[];
  C *lds = reinterpret_cast<C *>(circ_smem);
  __shared__ RunTables<Real> tabs[S::kSlots];
  __shared__ uint64_t alo[1 << kLowBits], ahi[1 << S::kHighBits];
  __shared__ uint32_t plo[1 << kLowBits], phi[1 << S::kHighBits];  // trailing swaps
  const uint32_t tid = threadIdx.x;
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  uint64_t base = 0;
  for (int b = 0; b < d.nfree; ++b) base |= (uint64_t)((tile >> b) & 1u) << pos_get(d.free_w, b);
  const int TL = d.TL, TH = d.T - d.TL;
  const uint32_t mlo = (1u << TL) - 1u;
  // element e of the tile is psi[alo[e & mlo] | ahi[e >> TL]]
  if (tid < 64u) {
    if (tid <= mlo) {
      uint64_t g = 0;
      uint32_t sp = 0;
      for (int q = 0; q < TL; ++q) {
        g |= (uint64_t)((tid >> q) & 1u) << pos_get(d.gpos_w, q);
        sp |= ((tid >> q) & 1u) << pos_get(d.perm_w, q);
      }
      alo[tid] = g;
      plo[tid] = sp;
    }
  } else if (tid - 64u < (1u << TH)) {
    const uint32_t j = tid - 64u;
    uint64_t g = base;
    uint32_t sp = 0;
    for (int q = 0; q < TH; ++q) {
      g |= (uint64_t)((j >> q) & 1u) << pos_get(d.gpos_w, TL + q);
      sp |= ((j >> q) & 1u) << pos_get(d.perm_w, TL + q);
    }
    ahi[j] = g;
    phi[j] = sp;
  }
  __syncthreads();
  const uint32_t TE = 1u << d.T;
  // the tile's loads, kLoadBatch per thread in flight before any LDS write
  for (uint32_t e0 = tid; e0 < TE; e0 += kLoadBatch * kCircThreads) {
    C t[kLoadBatch];
#pragma unroll
    for (int i = 0; i < kLoadBatch; ++i) {
      const uint32_t e = e0 + i * kCircThreads;
      if (e < TE) t[i] = psi[alo[e & mlo] | ahi[e >> TL]];
    }
#pragma unroll
    for (int i = 0; i < kLoadBatch; ++i) {
      const uint32_t e = e0 + i * kCircThreads;
      if (e < TE) lds[lidx(e)] = t[i];
    }
  }
  __syncthreads();
  int oi = 0;
  while (oi < d.nops) {
    const DevOp<Real> &op = ops[oi];
    const int kind = op.kind;
    if (kind == kOpStage) {
      const int cnt = op.a;
      if (op.nlo > 0) {  // the stage has diagonal runs: build their tables
        for (int i = 1; i <= cnt; ++i) {
          const DevOp<Real> &po = ops[oi + i];
          if (po.nlo + po.nhi + po.ncross > 0)
            build_tables<Real>(po, recs, tabs[po.slot], TL, TH, base, tid);
        }
        __syncthreads();
      }
      const uint32_t packed = (uint32_t)op.r0;
      if constexpr (FULL) {
        stage_sweep<Real, S::kStageBits>(lds, ops + oi + 1, cnt, packed, tabs, recs, base, TL,
                                         TE, tid);
      } else switch (op.b) {
        case 1: stage_sweep<Real, 1>(lds, ops + oi + 1, cnt, packed, tabs, recs, base, TL, TE, tid); break;
        case 2: stage_sweep<Real, 2>(lds, ops + oi + 1, cnt, packed, tabs, recs, base, TL, TE, tid); break;
        case 3: stage_sweep<Real, 3>(lds, ops + oi + 1, cnt, packed, tabs, recs, base, TL, TE, tid); break;
        case 4: stage_sweep<Real, 4>(lds, ops + oi + 1, cnt, packed, tabs, recs, base, TL, TE, tid); break;
        case 5:
          if constexpr (S::kStageBits >= 5)
            stage_sweep<Real, 5>(lds, ops + oi + 1, cnt, packed, tabs, recs, base, TL, TE, tid);
          break;
        default: break;
      }
      oi += 1 + cnt;
    } else {
      build_tables<Real>(op, recs, tabs[0], TL, TH, base, tid);
      __syncthreads();
      // each thread scales its elements e = tid + 256 i, kChunk at a time:
      // a per-element record is read once per chunk
      const int rc0 = op.r0 + op.nlo + op.nhi, rc1 = rc0 + op.ncross;
      for (uint32_t e0 = tid; e0 < TE; e0 += kChunk * kCircThreads) {
        C f[kChunk];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
          const uint32_t e = e0 + i * kCircThreads;
          f[i] = e < TE ? table_factor<Real>(tabs[0], e, TL, op.hx) : C{(Real)1, (Real)0};
        }
        for (int r = rc0; r < rc1; ++r) {
          const DevDiag<Real> rec = recs[r];
#pragma unroll
          for (int i = 0; i < kChunk; ++i)
            f[i] = cmul2(f[i], diag_factor(rec, e0 + i * kCircThreads, base));
        }
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
          const uint32_t e = e0 + i * kCircThreads;
          if (e < TE) lds[lidx(e)] = cmul2(f[i], lds[lidx(e)]);
        }
      }
      oi += 1;
    }
    __syncthreads();
  }
  // the trailing swaps: tile element e takes the element at plo | phi
  if (d.has_perm) {
    for (uint32_t e = tid; e < TE; e += kCircThreads)
      psi[alo[e & mlo] | ahi[e >> TL]] = lds[lidx(plo[e & mlo] | phi[e >> TL])];
  } else {
    for (uint32_t e = tid; e < TE; e += kCircThreads) psi[alo[e & mlo] | ahi[e >> TL]] = lds[lidx(e)];
  }
}

}  // namespace

struct qft_circuit_s {
  int n = 0;
  bool c128 = false;
  int device = 0;
  std::vector<GateRec> gates;
  // compiled form
  bool compiled = false;
  int tile_qubits = 0;
  std::vector<CircPass> passes;
  std::vector<int> gate_begin;  // first gate of each pass
  void *d_gates = nullptr;
};

namespace {

int check_qubit(const qft_circuit_s *c, int q) { return q >= 0 && q < c->n; }

void drop_compiled(qft_circuit_s *c) {
  if (c->d_gates) (void)hipFree(c->d_gates);
  c->d_gates = nullptr;
  c->passes.clear();
  c->gate_begin.clear();
  c->compiled = false;
}

int add_gate(qft_circuit_s *c, const GateRec &g) {
  try {
    c->gates.push_back(g);
  } catch (const std::bad_alloc &) {
    return set_error(QFT_ERR_NOMEM, "out of host memory");
  }
  if (c->compiled) drop_compiled(c);
  return QFT_OK;
}

bool is_diagonal(const GateRec &g) {
  return g.kind != kSwap && g.u[2] == 0.0 && g.u[3] == 0.0 && g.u[4] == 0.0 && g.u[5] == 0.0;
}

// The qubits a gate needs among the tile bits of its pass: the amplitudes it
// mixes.  A control, or any qubit of a diagonal gate, only selects or scales
// amplitudes, and its bit is known for every element from its global index.
std::vector<int> tile_needs(const GateRec &g) {
  if (g.kind == kSwap) return {g.a, g.b};
  if (is_diagonal(g)) return {};
  return {g.kind == kOne ? g.a : g.b};
}

int default_tile_bits(const qft_circuit_s *c) {
  return std::min(c->n, c->c128 ? kMaxTileC128 : kMaxTileC64);
}

// Device operations and diagonal records of one pass (host image).
template <typename Real>
struct PassImage {
  std::vector<DevOp<Real>> ops;
  std::vector<DevDiag<Real>> recs;
};

template <typename Real>
c2<Real> cval(const double *u, int i) {
  return c2<Real>{(Real)u[2 * i], (Real)u[2 * i + 1]};
}

template <typename Real>
void build_pass_image(const qft_circuit_s *c, int g0, int g1, const std::vector<int> &tpos,
                      int TL, PassImage<Real> &img, CircPass &pass) {
  // Swaps move no data: lab[q] is the LDS bit that holds logical tile
  // position q.  A swap of logical positions a and b maps state[e] to
  // state[P(e)], P exchanging bits a and b, so it exchanges lab[a] and
  // lab[b]; every later operand is a physical position, and the store
  // writes logical element e from the LDS element with bit lab[q] = bit q.
  std::vector<int> lab(pass.T);
  for (int q = 0; q < pass.T; ++q) lab[q] = q;
  auto enc = [&](int q) { return tpos[q] >= 0 ? lab[tpos[q]] : -1 - q; };
  std::vector<DevDiag<Real>> run;
  // Split a run of diagonal records over the low table (low positions,
  // global bits and the high position hx), the high table (high positions
  // and global bits) and the per-element list.  hx is the high position that
  // the most records pairing a low with a high position share (for the QFT,
  // the target of the run).
  auto flush = [&]() {
    if (run.empty()) return;
    auto is_low = [&](int32_t q) { return q >= 0 && q < TL; };
    auto is_high = [&](int32_t q) { return q >= TL; };
    std::vector<int> votes(64, 0);
    for (const DevDiag<Real> &r : run) {
      if (is_low(r.q1) && is_high(r.q0)) ++votes[r.q0];
      if (is_low(r.q0) && is_high(r.q1)) ++votes[r.q1];
    }
    int hx = -1;
    for (int q = 0; q < 64; ++q)
      if (votes[q] > 0 && (hx < 0 || votes[q] > votes[hx])) hx = q;
    std::vector<DevDiag<Real>> lo, hi, cross;
    for (const DevDiag<Real> &r : run) {
      const bool any_low = is_low(r.q1) || is_low(r.q0);
      const bool other_high = (is_high(r.q1) && r.q1 != hx) || (is_high(r.q0) && r.q0 != hx);
      if (!any_low) hi.push_back(r);
      else if (!other_high) lo.push_back(r);
      else cross.push_back(r);
    }
    // Each table entry multiplies all its table's records, and the two
    // tables are built side by side: records on global bits and hx only fit
    // either table, so move them to the low one until the counts balance.
    {
      auto movable = [&](const DevDiag<Real> &r) {
        return (r.q1 < 0 || r.q1 == hx) && (r.q0 < 0 || r.q0 == hx);
      };
      std::vector<DevDiag<Real>> stay;
      size_t nhi = hi.size();
      for (const DevDiag<Real> &r : hi) {
        if (movable(r) && lo.size() + 1 <= nhi - 1) {
          lo.push_back(r);
          --nhi;
        } else {
          stay.push_back(r);
        }
      }
      hi.swap(stay);
    }
    // the run rides on the pair operation just before it, if there is one
    const bool attach = !img.ops.empty() && img.ops.back().kind == kOpPair;
    if (!attach) {
      DevOp<Real> op;
      memset(&op, 0, sizeof(op));
      op.kind = kOpDiag;
      img.ops.push_back(op);
    }
    DevOp<Real> &op = img.ops.back();
    if (attach) {
      // anchored: every record involves the pair's target and scales only
      // amplitudes whose qubits are all 1
      const int32_t pos = op.a;
      const c2<Real> one{(Real)1, (Real)0};
      auto is_one = [&](const c2<Real> &z) { return z.x == one.x && z.y == one.y; };
      bool anchored = true;
      for (const DevDiag<Real> &r : run) {
        const bool ok = r.q1 == r.q0 ? (r.q0 == pos && is_one(r.D[0]))
                                     : ((r.q1 == pos || r.q0 == pos) && is_one(r.D[0]) &&
                                        is_one(r.D[1]) && is_one(r.D[2]));
        if (!ok) {
          anchored = false;
          break;
        }
      }
      if (anchored) {
        op.flags |= kAnchoredRun;
        op.apos = pos;
      }
    }
    op.r0 = (int32_t)img.recs.size();
    op.nlo = (int32_t)lo.size();
    op.nhi = (int32_t)hi.size();
    op.ncross = (int32_t)cross.size();
    op.hx = hx;
    img.recs.insert(img.recs.end(), lo.begin(), lo.end());
    img.recs.insert(img.recs.end(), hi.begin(), hi.end());
    img.recs.insert(img.recs.end(), cross.begin(), cross.end());
    run.clear();
  };
  const c2<Real> one{(Real)1, (Real)0};
  for (int i = g0; i < g1; ++i) {
    const GateRec &g = c->gates[i];
    if (is_diagonal(g)) {
      DevDiag<Real> r;
      memset(&r, 0, sizeof(r));
      if (g.kind == kOne) {
        r.q1 = r.q0 = enc(g.a);
        r.D[0] = cval<Real>(g.u, 0);
        r.D[1] = r.D[2] = one;  // unreachable: both bits are the same qubit
        r.D[3] = cval<Real>(g.u, 3);
      } else {
        r.q1 = enc(g.a);  // control
        r.q0 = enc(g.b);  // target
        r.D[0] = r.D[1] = one;
        r.D[2] = cval<Real>(g.u, 0);
        r.D[3] = cval<Real>(g.u, 3);
      }
      run.push_back(r);
      continue;
    }
    if (g.kind == kSwap) {
      // diagonal records already hold physical positions, so a run may
      // continue across the relabelling
      std::swap(lab[tpos[g.a]], lab[tpos[g.b]]);
      continue;
    }
    flush();
    DevOp<Real> op;
    memset(&op, 0, sizeof(op));
    op.hx = -1;  // no diagonal run (yet)
    op.kind = kOpPair;
    op.a = lab[tpos[g.kind == kOne ? g.a : g.b]];
    op.b = g.kind == kOne ? kNoControl : enc(g.a);
    for (int j = 0; j < 4; ++j) op.u[j] = cval<Real>(g.u, j);
    if (g.u[1] == 0.0 && g.u[3] == 0.0 && g.u[5] == 0.0 && g.u[7] == 0.0) op.flags |= kRealMatrix;
    img.ops.push_back(op);
  }
  flush();
  pass.has_perm = 0;
  for (int q = 0; q < pass.T; ++q) {
    pos_set(pass.perm_w, q, (uint32_t)lab[q]);
    if (lab[q] != q) pass.has_perm = 1;
  }
}

// Group consecutive pair operations into stages: greedily, while their
// targets span at most kStageBits tile positions and their diagonal runs fit
// the stage's table slots.  Each stage is a header followed by its pair
// operations, whose targets become indices into the stage's (ascending)
// positions.
//
// With T >= kStageBits every stage is padded to kStageBits positions with the
// highest tile positions it does not use (the extra positions only make each
// thread's sub-cube larger), so that the kernel needs one stage size only:
// its code then stays small enough for the instruction cache.
template <typename Real>
void form_stages(PassImage<Real> &img, int T) {
  const int kmax = Shape<Real>::kStageBits, slots = Shape<Real>::kSlots;
  std::vector<DevOp<Real>> out;
  size_t i = 0;
  while (i < img.ops.size()) {
    if (img.ops[i].kind != kOpPair) {
      out.push_back(img.ops[i]);
      ++i;
      continue;
    }
    std::vector<int> S;
    int runs = 0;
    size_t j = i;
    while (j < img.ops.size() && img.ops[j].kind == kOpPair) {
      const DevOp<Real> &o = img.ops[j];
      const bool run = o.nlo + o.nhi + o.ncross > 0;
      const bool fresh = std::find(S.begin(), S.end(), o.a) == S.end();
      if ((fresh && (int)S.size() == kmax) || (run && runs == slots)) break;
      if (fresh) S.push_back(o.a);
      if (run) ++runs;
      ++j;
    }
    for (int q = T - 1; q >= 0 && T >= kmax && (int)S.size() < kmax; --q)
      if (std::find(S.begin(), S.end(), q) == S.end()) S.push_back(q);
    std::sort(S.begin(), S.end());
    DevOp<Real> h;
    memset(&h, 0, sizeof(h));
    h.kind = kOpStage;
    h.a = (int32_t)(j - i);
    h.b = (int32_t)S.size();
    uint32_t packed = 0;
    for (size_t q = 0; q < S.size(); ++q) packed |= (uint32_t)S[q] << (4 * q);
    h.r0 = (int32_t)packed;
    h.nlo = runs;
    h.hx = -1;
    out.push_back(h);
    int slot = 0;
    for (size_t k = i; k < j; ++k) {
      DevOp<Real> o = img.ops[k];
      o.a = (int32_t)(std::find(S.begin(), S.end(), o.a) - S.begin());
      if (o.nlo + o.nhi + o.ncross > 0) o.slot = slot++;
      out.push_back(o);
    }
    i = j;
  }
  img.ops.swap(out);
}

template <typename Real>
int upload_passes(qft_circuit_s *c, std::vector<PassImage<Real>> &imgs) {
  size_t bytes = 0;
  std::vector<size_t> off_ops(imgs.size()), off_recs(imgs.size());
  for (size_t r = 0; r < imgs.size(); ++r) {
    off_ops[r] = bytes;
    bytes += imgs[r].ops.size() * sizeof(DevOp<Real>);
    off_recs[r] = bytes;
    bytes += imgs[r].recs.size() * sizeof(DevDiag<Real>);
  }
  std::vector<unsigned char> host(bytes);
  for (size_t r = 0; r < imgs.size(); ++r) {
    if (!imgs[r].ops.empty())
      memcpy(host.data() + off_ops[r], imgs[r].ops.data(),
             imgs[r].ops.size() * sizeof(DevOp<Real>));
    if (!imgs[r].recs.empty())
      memcpy(host.data() + off_recs[r], imgs[r].recs.data(),
             imgs[r].recs.size() * sizeof(DevDiag<Real>));
  }
  if (bytes) {
    hipError_t e = hipMalloc(&c->d_gates, bytes);
    if (e != hipSuccess) {
      c->d_gates = nullptr;
      return hip_error(e, "circuit gate upload");
    }
    e = hipMemcpy(c->d_gates, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "circuit gate upload");
  }
  for (size_t r = 0; r < imgs.size(); ++r) {
    c->passes[r].ops = (unsigned char *)c->d_gates + off_ops[r];
    c->passes[r].recs = (unsigned char *)c->d_gates + off_recs[r];
  }
  return QFT_OK;
}

int compile(qft_circuit_s *c, int tile_qubits, bool upload) {
  drop_compiled(c);
  const int n = c->n;
  const int T = default_tile_bits(c);
  // by default leave 64 bytes of contiguous elements per tile row (the
  // passes are bound by their LDS sweeps more than by row length)
  int B = tile_qubits > 0 ? tile_qubits : T - (c->c128 ? 2 : 3);
  B = std::max(2, std::min(B, T));
  c->tile_qubits = tile_qubits;
  // greedy runs of gates whose tile needs fit in B qubits
  std::vector<std::pair<int, int>> runs;
  std::vector<std::vector<int>> sets;
  {
    std::vector<int> S;
    int start = 0;
    for (int i = 0; i < (int)c->gates.size(); ++i) {
      const std::vector<int> need = tile_needs(c->gates[i]);
      std::vector<int> U = S;
      for (int q : need)
        if (std::find(U.begin(), U.end(), q) == U.end()) U.push_back(q);
      if ((int)U.size() > B) {
        runs.push_back({start, i});
        sets.push_back(S);
        start = i;
        U = need;
        std::sort(U.begin(), U.end());
        U.erase(std::unique(U.begin(), U.end()), U.end());
      }
      S = U;
    }
    if (!c->gates.empty()) {
      runs.push_back({start, (int)c->gates.size()});
      sets.push_back(S);
    }
  }
  std::vector<PassImage<float>> img32;
  std::vector<PassImage<double>> img64;
  for (size_t r = 0; r < runs.size(); ++r) {
    // tile: the run's needed qubits plus the lowest other qubits, up to T
    // bits, ordered by global bit so that low tile bits give contiguous rows
    std::vector<int> tile = sets[r];
    for (int q = 0; q < n && (int)tile.size() < T; ++q)
      if (std::find(tile.begin(), tile.end(), q) == tile.end()) tile.push_back(q);
    std::sort(tile.begin(), tile.end());
    std::vector<int> tpos(n, -1);
    CircPass p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.T = (int)tile.size();
    p.TL = std::min(p.T, kLowBits);
    for (int q = 0; q < p.T; ++q) {
      pos_set(p.gpos_w, q, (uint32_t)tile[q]);
      tpos[tile[q]] = q;
    }
    int nf = 0;
    for (int b = 0; b < n; ++b)
      if (tpos[b] < 0) pos_set(p.free_w, nf++, (uint32_t)b);
    p.nfree = nf;
    p.ntiles = 1u << nf;
    p.xcd_remap = (p.ntiles >= 8 && p.ntiles % 8 == 0) ? 1 : 0;
    if (c->c128) {
      img64.emplace_back();
      build_pass_image<double>(c, runs[r].first, runs[r].second, tpos, p.TL, img64.back(), p);
      form_stages<double>(img64.back(), p.T);
      p.nops = (int)img64.back().ops.size();
    } else {
      img32.emplace_back();
      build_pass_image<float>(c, runs[r].first, runs[r].second, tpos, p.TL, img32.back(), p);
      form_stages<float>(img32.back(), p.T);
      p.nops = (int)img32.back().ops.size();
    }
    c->passes.push_back(p);
    c->gate_begin.push_back(runs[r].first);
  }
  if (!upload) return QFT_OK;  // host grouping only (describe)
  const int rc = c->c128 ? upload_passes<double>(c, img64) : upload_passes<float>(c, img32);
  if (rc != QFT_OK) return rc;
  c->compiled = true;
  return QFT_OK;
}

template <typename Real>
constexpr int kMaxTile() {
  return sizeof(Real) == 8 ? kMaxTileC128 : kMaxTileC64;
}

// Dynamic LDS of a pass: the tile with one pad element per 32 (see lidx).
template <typename Real>
size_t circuit_lds_bytes(int T) {
  const size_t te = (size_t)1 << T;
  return (te + (te >> 5)) * sizeof(c2<Real>);
}

template <typename Real>
hipError_t launch_circuit_pass(const CircPass &p, void *dev_ptr, hipStream_t s) {
  const size_t lds = circuit_lds_bytes<Real>(p.T);
  auto fn = p.T >= Shape<Real>::kStageBits ? k_circuit_pass<Real, true>
                                           : k_circuit_pass<Real, false>;
  if (lds > 65536) {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void *>(fn),
                                    (int)circuit_lds_bytes<Real>(kMaxTile<Real>()));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(p.ntiles), dim3(kCircThreads), lds, s, p, (c2<Real> *)dev_ptr,
                     (const DevOp<Real> *)p.ops, (const DevDiag<Real> *)p.recs);
  return hipGetLastError();
}

}  // namespace

extern "C" {

qft_circuit_t *qft_circuit_create(int n, int layout) {
  clear_error();
  if (n < 1 || n > QFT_MAX_QUBITS) {
    set_error(QFT_ERR_INVALID, "n out of range");
    return nullptr;
  }
  qft_circuit_s *c = new (std::nothrow) qft_circuit_s();
  if (!c) {
    set_error(QFT_ERR_NOMEM, "out of host memory");
    return nullptr;
  }
  c->n = n;
  c->c128 = (layout & QFT_C128) != 0;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  return c;
}

void qft_circuit_destroy(qft_circuit_t *c) {
  if (!c) return;
  drop_compiled(c);
  delete c;
}

int qft_circuit_add_1q(qft_circuit_t *c, int q, const double u[8]) {
  clear_error();
  if (!c || !u) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!check_qubit(c, q)) return set_error(QFT_ERR_INVALID, "qubit out of range");
  GateRec g;
  g.kind = kOne;
  g.a = q;
  g.b = -1;
  memcpy(g.u, u, sizeof(g.u));
  return add_gate(c, g);
}

int qft_circuit_add_controlled(qft_circuit_t *c, int control, int target, const double u[8]) {
  clear_error();
  if (!c || !u) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!check_qubit(c, control) || !check_qubit(c, target) || control == target)
    return set_error(QFT_ERR_INVALID, "bad control / target qubits");
  GateRec g;
  g.kind = kControlled;
  g.a = control;
  g.b = target;
  memcpy(g.u, u, sizeof(g.u));
  return add_gate(c, g);
}

int qft_circuit_add_swap(qft_circuit_t *c, int a, int b) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!check_qubit(c, a) || !check_qubit(c, b) || a == b)
    return set_error(QFT_ERR_INVALID, "bad swap qubits");
  GateRec g;
  memset(&g, 0, sizeof(g));
  g.kind = kSwap;
  g.a = a;
  g.b = b;
  return add_gate(c, g);
}

int qft_circuit_compile(qft_circuit_t *c, int tile_qubits) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (tile_qubits < 0) return set_error(QFT_ERR_INVALID, "tile_qubits < 0");
  return compile(c, tile_qubits, true);
}

int qft_circuit_describe(qft_circuit_t *c, int tile_qubits, int *gate_begin, int *tile_bits,
                         int max_passes) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (tile_qubits < 0) return set_error(QFT_ERR_INVALID, "tile_qubits < 0");
  const int keep = c->tile_qubits;
  int rc = compile(c, tile_qubits, false);
  c->tile_qubits = keep;
  if (rc != QFT_OK) return rc;
  const int np = (int)c->passes.size();
  for (int i = 0; i < np && i < max_passes; ++i) {
    if (gate_begin) gate_begin[i] = c->gate_begin[i];
    if (tile_bits) tile_bits[i] = c->passes[i].T;
  }
  drop_compiled(c);
  return np;
}

int qft_circuit_info(const qft_circuit_t *c, int *gates, int *passes) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (gates) *gates = (int)c->gates.size();
  if (passes) *passes = c->compiled ? (int)c->passes.size() : -1;
  return QFT_OK;
}

int qft_circuit_execute(qft_circuit_t *c, void *dev_ptr, qft_stream_t stream) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (!dev_ptr) return set_error(QFT_ERR_POINTER, "data pointer is NULL");
  if ((uintptr_t)dev_ptr % (c->c128 ? 16 : 8))
    return set_error(QFT_ERR_POINTER, "data pointer is not aligned to the element size");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return set_error(QFT_ERR_INVALID, "the current device is not the circuit's device");
  if (!c->compiled) {
    int rc = compile(c, c->tile_qubits, true);
    if (rc != QFT_OK) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  for (const CircPass &p : c->passes) {
    hipError_t e = c->c128 ? launch_circuit_pass<double>(p, dev_ptr, s)
                           : launch_circuit_pass<float>(p, dev_ptr, s);
    if (e != hipSuccess) return hip_error(e, "circuit pass launch");
  }
  return QFT_OK;
}

}  // extern "C"
