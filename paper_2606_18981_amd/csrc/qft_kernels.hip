// gfx950 kernels of the QFT->FFT path.
//
// k_fused_pass: one HBM pass of the fused schedule.  A workgroup owns one
//   tile of 2^T elements (m pass bits + spectator bits, see qft_internal.h).
//   Each thread holds R = 2^RB elements in registers; the pass bits are
//   applied RB at a time (radix-2^RB decimation-in-frequency in registers),
//   with an LDS exchange between register groups.  Per target qubit t the
//   work is the circuit's H(t) (Fig. 1) - here an unnormalised butterfly, the
//   1/sqrt(2) factors being folded into one per-pass scale - followed by the
//   product of the controlled phases of target t whose control lies inside
//   the pass (Sec. 2: that product is the FFT twiddle T~).  Controlled
//   phases whose control lies below the pass are applied as one diagonal at
//   the end of the pass.  The last pass writes bit-reversed addresses when the
//   final swaps are requested (Sec. 3 step 2).
// k_h / k_cphase / k_swap: the unfused circuit, one sweep per gate.
// k_fill_random: Philox-4x32-10 (Salmon et al., SC 2011) counter-based input
//   generator with FP64 Box-Muller.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <set>
#include <utility>

#include "qft_internal.h"
#include "qft_kernels.h"

namespace qft {

hipError_t ensure_lds_limit(const void *fn, int bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  static std::mutex mu;
  static std::set<std::pair<int, const void *>> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({dev, fn})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  done.insert({dev, fn});
  return hipSuccess;
}


template <typename Real>
struct alignas(2 * sizeof(Real)) cplx {
  Real x, y;
};

template <typename Real>
__device__ __forceinline__ cplx<Real> cadd(cplx<Real> a, cplx<Real> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename Real>
__device__ __forceinline__ cplx<Real> csub(cplx<Real> a, cplx<Real> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename Real>
__device__ __forceinline__ cplx<Real> cmul(cplx<Real> a, cplx<Real> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ uint32_t rev_bits(uint32_t x, int n) {
  return __builtin_bitreverse32(x) >> (32 - n);
}

// LDS slot of tile element e: the low SW bits are XORed with a fold of the
// higher bits.  The map is linear over GF(2) (and a bijection), so the slot of
// e_thr | e_reg is slot(e_thr) ^ slot(e_reg): one XOR per element against a
// wave-uniform term.
template <typename Real>
__host__ __device__ __forceinline__ uint32_t lds_swizzle(uint32_t e) {
  constexpr int SW = sizeof(Real) == 4 ? 4 : 3;
  const uint32_t h = (e >> SW) ^ (e >> (2 * SW)) ^ (e >> (3 * SW)) ^ (e >> (4 * SW));
  return e ^ (h & ((1u << SW) - 1u));
}

__device__ __forceinline__ uint32_t deposit_tid(uint32_t tid, const uint32_t *pos, int nb) {
  uint32_t e = 0;
  for (int b = 0; b < nb; ++b) e |= ((tid >> b) & 1u) << pos_get(pos, b);
  return e;
}

template <int RB>
__device__ __forceinline__ uint32_t deposit_reg(int rho, const uint32_t *pos) {
  uint32_t o = 0;
#pragma unroll
  for (int q = 0; q < RB; ++q)
    if ((rho >> q) & 1) o |= 1u << pos_get(pos, q);
  return o;
}

// cos(2 pi j / 32), j = 0..8
__device__ constexpr double kCos32[9] = {
    1.0, 0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
    0.70710678118654752440, 0.55557023301960222474, 0.38268343236508977173,
    0.19509032201612826785, 0.0};

// z * w_32^J with w_32 = exp(-2 pi i / 32), 0 <= J < 16 (J is a constant after
// unrolling, so the branches fold away).
template <typename Real>
__device__ __forceinline__ cplx<Real> mul_w32(cplx<Real> z, int J) {
  if (J == 0) return z;
  if (J == 8) return {z.y, -z.x};  // -i
  const Real h = (Real)0.70710678118654752440;
  if (J == 4) return {(z.x + z.y) * h, (z.y - z.x) * h};
  if (J == 12) return {(z.y - z.x) * h, -(z.x + z.y) * h};
  // w_32^J = c - i s with c = cos(2 pi J/32), s = sin(2 pi J/32)
  const Real c = J <= 8 ? (Real)kCos32[J] : -(Real)kCos32[16 - J];
  const Real sn = J <= 8 ? (Real)kCos32[8 - J] : (Real)kCos32[J - 8];
  return {z.x * c + z.y * sn, z.y * c - z.x * sn};
}

// Radix-2^nst decimation-in-frequency network on register bits nst-1 .. 0:
// for target register bit q the butterfly (a, b) -> (a + b, (a - b) w) with
// the twiddle w = w_{2^{q+1}}^{rho mod 2^q} of the controlled phases whose
// controls are the register bits below q.  Controls held by other threads are
// applied afterwards by apply_factors (they commute with these butterflies).
template <typename Real, int RB>
__device__ __forceinline__ void radix_network(cplx<Real> (&v)[1 << RB], int nst) {
  constexpr int R = 1 << RB;
#pragma unroll
  for (int q = RB - 1; q >= 0; --q) {
    if (q < nst) {
#pragma unroll
      for (int rho = 0; rho < R; ++rho) {
        if (rho & (1 << q)) continue;
        const int hi = rho | (1 << q);
        const cplx<Real> a = v[rho];
        const cplx<Real> b = v[hi];
        v[rho] = cadd(a, b);
        v[hi] = mul_w32(csub(a, b), (rho & ((1 << q) - 1)) << (4 - q));
      }
    }
  }
}

// v[rho] *= F(rho), F(rho) = f0 * prod_{q : bit q of rho set} f[q].  The
// products are built separately for the low and the high half of the register
// bits (two small subset-product tables), so that about two complex
// multiplies per element suffice and few registers stay live.  With
// apply0 == false, f0 is taken as 1.
template <typename Real, int RB>
__device__ __forceinline__ void apply_factors(cplx<Real> (&v)[1 << RB], const cplx<Real> (&f)[RB],
                                              cplx<Real> f0, bool apply0) {
  constexpr int R = 1 << RB;
  constexpr int SL = RB / 2;
  constexpr int NL = 1 << SL;
  constexpr int NH = 1 << (RB - SL);
  cplx<Real> Fl[NL], Fh[NH];
  Fl[0] = f0;
#pragma unroll
  for (int a = 1; a < NL; ++a) {
    const int top = 31 - __builtin_clz(a);
    const int rest = a & ~(1 << top);
    Fl[a] = (rest == 0 && !apply0) ? f[top] : cmul(Fl[rest], f[top]);
  }
  Fh[0] = cplx<Real>{(Real)1, (Real)0};
#pragma unroll
  for (int b = 1; b < NH; ++b) {
    const int top = 31 - __builtin_clz(b);
    const int rest = b & ~(1 << top);
    Fh[b] = rest == 0 ? f[SL + top] : cmul(Fh[rest], f[SL + top]);
  }
#pragma unroll
  for (int rho = 0; rho < R; ++rho) {
    const int a = rho & (NL - 1);
    const int b = rho >> SL;
    if (b == 0) {
      if (a != 0 || apply0) v[rho] = cmul(v[rho], Fl[a]);
    } else if (a == 0 && !apply0) {
      v[rho] = cmul(v[rho], Fh[b]);
    } else {
      v[rho] = cmul(v[rho], cmul(Fl[a], Fh[b]));
    }
  }
}

// The same product in two steps: every element is multiplied by its
// low-half subset factor, then by its high-half one.  Two complex multiplies
// per element, as in apply_factors, but only one subset table is live at a
// time: the four-wave kernels (128 VGPRs per lane) need the registers.
template <typename Real, int RB>
__device__ __forceinline__ void apply_factors_lean(cplx<Real> (&v)[1 << RB],
                                                   const cplx<Real> (&f)[RB], cplx<Real> f0,
                                                   bool apply0) {
  constexpr int R = 1 << RB;
  constexpr int SL = RB / 2;
  constexpr int NL = 1 << SL;
  constexpr int NH = 1 << (RB - SL);
  {
    cplx<Real> Fl[NL];
    Fl[0] = f0;
#pragma unroll
    for (int a = 1; a < NL; ++a) {
      const int top = 31 - __builtin_clz(a);
      const int rest = a & ~(1 << top);
      Fl[a] = (rest == 0 && !apply0) ? f[top] : cmul(Fl[rest], f[top]);
    }
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
      const int a = rho & (NL - 1);
      if (a != 0 || apply0) v[rho] = cmul(v[rho], Fl[a]);
    }
  }
  cplx<Real> Fh[NH];
  Fh[0] = cplx<Real>{(Real)1, (Real)0};
#pragma unroll
  for (int b = 1; b < NH; ++b) {
    const int top = 31 - __builtin_clz(b);
    const int rest = b & ~(1 << top);
    Fh[b] = rest == 0 ? f[SL + top] : cmul(Fh[rest], f[SL + top]);
  }
#pragma unroll
  for (int rho = 0; rho < R; ++rho) {
    const int b = rho >> SL;
    if (b != 0) v[rho] = cmul(v[rho], Fh[b]);
  }
}

// Subset-product factors: the four-wave kernels (W4) take the two-step form.
template <typename Real, int RB, bool W4>
__device__ __forceinline__ void apply_factors_k(cplx<Real> (&v)[1 << RB], const cplx<Real> (&f)[RB],
                                                cplx<Real> f0, bool apply0) {
  if constexpr (W4) apply_factors_lean<Real, RB>(v, f, f0, apply0);
  else apply_factors<Real, RB>(v, f, f0, apply0);
}

// Index of the tile's first element: the tile number deposited into the
// non-tile bit positions.
__device__ __forceinline__ uint32_t tile_base(const PassDesc &d, uint32_t tile) {
  uint32_t base = 0;
  for (int b = 0; b < d.nfree; ++b) base |= ((tile >> b) & 1u) << pos_get(d.free_w, b);
  return base;
}

// Controls among this thread's pass bits below jbase: target jl = jbase + q
// gets w_{2^{jl+1}}^{u} on elements with register bit q set, u = those bits
// with the ones below jl - k cleared (AQFT).  Depends on the thread only, not
// on the tile.
template <typename Real, int RB>
__device__ __forceinline__ void group_factors(const PassDesc &d, const GroupMap &G, uint32_t e_thr,
                                              cplx<Real> (&f)[RB]) {
  const cplx<Real> *__restrict__ W = (const cplx<Real> *)d.tw_int;
  const int MI1 = d.MI - 1;
  const int jbase = G.jbase;
  const uint32_t u_thr = (e_thr >> d.pbase) & ((1u << jbase) - 1u);
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int jl = jbase + q;
    int clear = d.aqft ? jl - d.k : 0;
    clear = clear < 0 ? 0 : clear;
    const uint32_t x = clear >= jbase ? 0u : ((u_thr >> clear) << clear);
    f[q] = q < G.nst ? W[x << (MI1 - jl)] : cplx<Real>{(Real)1, (Real)0};
  }
}

// Diagonal of the controlled phases whose controls lie below the pass:
// w_N^E with E = sum over set pass bits j of trunc_{lo+j-k}(vv) 2^{n-1-lo-j}
// (vv = index bits below the pass).  All register bits of the store map are
// pass bits, so E = E_thr + sum over set register bits q of c_q: the factors
// are f0 = w_N^{E_thr} (times the pass scale) and f[q] = w_N^{c_q}.  Each is
// the product of a low-table and a high-table entry.  ext_loads issues the
// table reads (g = index of the thread's register-0 element); ext_finish
// multiplies them, so that the reads can be in flight with the tile's own.
template <typename Real, int RB>
struct ExtRaw {
  cplx<Real> lo[RB + 1], hi[RB + 1];  // [RB] is f0's pair
};

template <typename Real, int RB>
__device__ __forceinline__ void ext_loads(const PassDesc &d, uint32_t g, ExtRaw<Real, RB> &raw) {
  const cplx<Real> *__restrict__ tlo = (const cplx<Real> *)d.tw_lo;
  const cplx<Real> *__restrict__ thi = (const cplx<Real> *)d.tw_hi;
  const uint32_t nmask = d.n >= 32 ? 0xffffffffu : ((1u << d.n) - 1u);
  const uint32_t lmask = (1u << d.L) - 1u;
  const uint32_t vv = g & ((1u << d.lo) - 1u);
  const uint32_t pt = (g >> d.lo) & ((1u << d.m) - 1u);
  uint32_t Et = 0;
  if (!d.aqft) {
    Et = (vv * rev_bits(pt, d.m)) << (d.n - d.lo - d.m);
  } else {
    for (int j = 0; j < d.m; ++j) {
      if ((pt >> j) & 1u) {
        const int s = d.lo + j - d.k;
        const uint32_t tv = s <= 0 ? vv : (s >= d.lo ? 0u : ((vv >> s) << s));
        Et = (Et + (tv << (d.n - 1 - d.lo - j))) & nmask;
      }
    }
  }
  raw.lo[RB] = tlo[Et & lmask];
  raw.hi[RB] = thi[Et >> d.L];
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int j = (int)pos_get(d.st_reg_w, q) - d.lo;
    const int s = d.lo + j - d.k;
    const uint32_t tv = (!d.aqft || s <= 0) ? vv : (s >= d.lo ? 0u : ((vv >> s) << s));
    const uint32_t E = (tv << (d.n - 1 - d.lo - j)) & nmask;
    raw.lo[q] = tlo[E & lmask];
    raw.hi[q] = thi[E >> d.L];
  }
}

template <typename Real, int RB>
__device__ __forceinline__ void ext_finish(const PassDesc &d, const ExtRaw<Real, RB> &raw,
                                           cplx<Real> (&f)[RB], cplx<Real> &f0) {
#pragma unroll
  for (int q = 0; q < RB; ++q) f[q] = cmul(raw.lo[q], raw.hi[q]);
  f0 = cmul(raw.lo[RB], raw.hi[RB]);
  const Real scale = (Real)d.scale;
  f0.x *= scale;
  f0.y *= scale;
}

// Move the registers from group P's map to group G's map through LDS.
template <typename Real, int RB>
__device__ __forceinline__ void exchange(cplx<Real> (&v)[1 << RB], cplx<Real> *lds,
                                         const GroupMap &P, const GroupMap &G, uint32_t tid, int TR,
                                         bool active) {
  constexpr int R = 1 << RB;
  if (active) {
    const uint32_t sp = lds_swizzle<Real>(deposit_tid(tid, P.thr_w, TR));
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
      lds[sp ^ lds_swizzle<Real>(deposit_reg<RB>(rho, P.reg_w))] = v[rho];
  }
  __syncthreads();
  if (active) {
    const uint32_t sg = lds_swizzle<Real>(deposit_tid(tid, G.thr_w, TR));
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
      v[rho] = lds[sg ^ lds_swizzle<Real>(deposit_reg<RB>(rho, G.reg_w))];
  }
  __syncthreads();
}

// The same exchange in two halves: real parts, then imaginary parts, through
// an LDS area of 2^T scalars (half the tile).  Four barriers instead of two,
// but half the LDS per workgroup, so three 2^13-element complex64 workgroups
// fit a CU's 160 KiB instead of two.  Slots are the tile positions
// themselves: with 4-byte slots the XOR fold measured slower (2.64-2.67 ms
// against 2.61 ms at 2^28).
//
// FENCE: the four-wave kernels keep the compiler from computing the LDS
// addresses of all four phases up front (64 of them would be live at once,
// and with the 64 data registers the 128-VGPR budget spills).
template <typename Real, int RB, bool FENCE = false>
__device__ __forceinline__ void exchange_split(cplx<Real> (&v)[1 << RB], cplx<Real> *lds_c,
                                               const GroupMap &P, const GroupMap &G,
                                               uint32_t tid, int TR) {
  constexpr int R = 1 << RB;
  Real *lds = reinterpret_cast<Real *>(lds_c);
  const uint32_t sp = deposit_tid(tid, P.thr_w, TR);
  const uint32_t sg = deposit_tid(tid, G.thr_w, TR);
#pragma unroll
  for (int rho = 0; rho < R; ++rho)
    lds[sp | deposit_reg<RB>(rho, P.reg_w)] = v[rho].x;
  __syncthreads();
  if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int rho = 0; rho < R; ++rho)
    v[rho].x = lds[sg | deposit_reg<RB>(rho, G.reg_w)];
  __syncthreads();
  if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int rho = 0; rho < R; ++rho)
    lds[sp | deposit_reg<RB>(rho, P.reg_w)] = v[rho].y;
  __syncthreads();
  if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int rho = 0; rho < R; ++rho)
    v[rho].y = lds[sg | deposit_reg<RB>(rho, G.reg_w)];
  __syncthreads();
}

template <typename Real, int RB>
__device__ __forceinline__ void conj_regs(cplx<Real> (&v)[1 << RB]) {
#pragma unroll
  for (int rho = 0; rho < (1 << RB); ++rho) v[rho].y = -v[rho].y;
}

// One element load / store; NT selects the non-temporal (streaming) form.
template <bool NT, typename Real>
__device__ __forceinline__ cplx<Real> ld_elem(const cplx<Real> *p) {
  if constexpr (NT) {
    typedef Real V2 __attribute__((ext_vector_type(2)));
    const V2 t = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(p));
    return cplx<Real>{t.x, t.y};
  } else {
    return *p;
  }
}
template <bool NT, typename Real>
__device__ __forceinline__ void st_elem(cplx<Real> *p, cplx<Real> v) {
  if constexpr (NT) {
    typedef Real V2 __attribute__((ext_vector_type(2)));
    const V2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<V2 *>(p));
  } else {
    *p = v;
  }
}

// Branch-free conjugation: flip the sign bit of every imaginary part when
// `on` (no data-dependent control flow, so no register merges).
template <int RB>
__device__ __forceinline__ void conj_if(cplx<float> (&v)[1 << RB], bool on) {
  const uint32_t m = on ? 0x80000000u : 0u;
#pragma unroll
  for (int rho = 0; rho < (1 << RB); ++rho) v[rho].y = __uint_as_float(__float_as_uint(v[rho].y) ^ m);
}
template <int RB>
__device__ __forceinline__ void conj_if(cplx<double> (&v)[1 << RB], bool on) {
  const uint64_t m = on ? 0x8000000000000000ull : 0ull;
#pragma unroll
  for (int rho = 0; rho < (1 << RB); ++rho)
    v[rho].y = __longlong_as_double((long long)((uint64_t)__double_as_longlong(v[rho].y) ^ m));
}

template <typename Real, int RB, bool NT>
__device__ __forceinline__ void store_tile_raw(const PassDesc &d, const cplx<Real> (&v)[1 << RB],
                                               cplx<Real> *dst) {
  constexpr int R = 1 << RB;
  uint32_t soff[R];
#pragma unroll
  for (int rho = 0; rho < R; ++rho) soff[rho] = deposit_reg<RB>(rho, d.st_reg_w);
#pragma unroll
  for (int rho = 0; rho < R; ++rho) st_elem<NT>(dst + soff[rho], v[rho]);
}

template <typename Real, int RB>
__device__ __forceinline__ void store_tile(const PassDesc &d, cplx<Real> (&v)[1 << RB],
                                           cplx<Real> *dst) {
  constexpr int R = 1 << RB;
  if (d.conj_out) conj_regs<Real, RB>(v);
  uint32_t soff[R];
#pragma unroll
  for (int rho = 0; rho < R; ++rho) soff[rho] = deposit_reg<RB>(rho, d.st_reg_w);
#pragma unroll
  for (int rho = 0; rho < R; ++rho) dst[soff[rho]] = v[rho];
}

// Sum of |x|^2 over the tile's loaded elements, one partial per wave (or per
// thread when the workgroup is smaller than a wave), accumulated in FP64.
// Every thread of the workgroup calls it (inactive ones hold zeros).
template <typename Real, int RB>
__device__ __forceinline__ void norm_partial(const cplx<Real> (&v)[1 << RB], double *part,
                                             uint32_t tile, uint32_t tid) {
  double a = 0.0;
#pragma unroll
  for (int rho = 0; rho < (1 << RB); ++rho) a += (double)(v[rho].x * v[rho].x + v[rho].y * v[rho].y);
  const uint32_t threads = blockDim.x;
  if (threads >= 64) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((tid & 63u) == 0) part[(size_t)tile * (threads >> 6) + (tid >> 6)] = a;
  } else {
    part[(size_t)tile * threads + tid] = a;
  }
}

// One tile of one pass.  Per register group: radix network on the group's
// register bits, then the controlled phases whose controls are this thread's
// lower pass bits (deferred to the end of the group), then an LDS exchange to
// the next group's mapping.  At the end: the diagonal of the controls below
// the pass (high passes), the folded scale, and the store (bit-reversed
// addresses in the final pass of a natural-order plan).  The twiddle-table
// reads of the first two groups and of the final diagonal are issued before
// the tile's loads, so the tile waits for one memory latency, not one per
// table.  Threads with active == false (workgroups larger than the tile
// needs) only take part in the barriers.
template <typename Real, int RB>
__device__ __forceinline__ void tile_body(const PassDesc &d, uint32_t tile, const cplx<Real> *in,
                                          cplx<Real> *out, cplx<Real> *lds, uint32_t tid,
                                          bool active) {
  using C = cplx<Real>;
  constexpr int R = 1 << RB;
  const int TR = d.T - RB;
  const uint32_t base = tile_base(d, tile);
  const uint32_t st_thr = deposit_tid(tid, d.st_thr_w, TR);

  const bool has0 = d.ngroups > 0 && d.grp[0].jbase > 0 && d.grp[0].nst > 0;
  const bool has1 = d.ngroups > 1 && d.grp[1].jbase > 0 && d.grp[1].nst > 0;
  C gf0[RB], gf1[RB];
  ExtRaw<Real, RB> raw;
  if (active) {
    if (has0) group_factors<Real, RB>(d, d.grp[0], deposit_tid(tid, d.grp[0].thr_w, TR), gf0);
    if (has1) group_factors<Real, RB>(d, d.grp[1], deposit_tid(tid, d.grp[1].thr_w, TR), gf1);
    if (d.ext_tw) ext_loads<Real, RB>(d, base | st_thr, raw);
  }

  C v[R];
  if (active) {
    const C *src = in + (base | deposit_tid(tid, d.ld_thr_w, TR));
#pragma unroll
    for (int rho = 0; rho < R; ++rho) v[rho] = src[deposit_reg<RB>(rho, d.ld_reg_w)];
    if (d.conj_in) conj_regs<Real, RB>(v);
  } else {
#pragma unroll
    for (int rho = 0; rho < R; ++rho) v[rho] = C{(Real)0, (Real)0};
  }
  if (d.norm_part) norm_partial<Real, RB>(v, d.norm_part, tile, tid);

  radix_network<Real, RB>(v, d.grp[0].nst);
  if (has0 && active) apply_factors<Real, RB>(v, gf0, C{(Real)1, (Real)0}, false);
  for (int gi = 1; gi < d.ngroups; ++gi) {
    const GroupMap &G = d.grp[gi];
    exchange<Real, RB>(v, lds, d.grp[gi - 1], G, tid, TR, active);
    radix_network<Real, RB>(v, G.nst);
    if (gi == 1) {
      if (has1 && active) apply_factors<Real, RB>(v, gf1, C{(Real)1, (Real)0}, false);
    } else if (G.jbase > 0 && G.nst > 0 && active) {
      C f[RB];
      group_factors<Real, RB>(d, G, deposit_tid(tid, G.thr_w, TR), f);
      apply_factors<Real, RB>(v, f, C{(Real)1, (Real)0}, false);
    }
  }
  if (!active) return;

  const uint32_t obase = d.reverse ? rev_bits(base, d.n) : base;
  if (d.ext_tw) {
    C f[RB], f0;
    ext_finish<Real, RB>(d, raw, f, f0);
    apply_factors<Real, RB>(v, f, f0, true);
  } else {
    const Real scale = (Real)d.scale;
    if (scale != (Real)1) {
#pragma unroll
      for (int rho = 0; rho < R; ++rho) {
        v[rho].x *= scale;
        v[rho].y *= scale;
      }
    }
  }
  store_tile<Real, RB>(d, v, out + (obase | st_thr));
}

template <typename Real, int RB>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? (RB >= 5 ? 256 : RB >= 3 ? 512 : 1024)
                                                   : (RB >= 5 ? 512 : 1024))
k_fused_pass(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    // consecutive tiles on one XCD (workgroups are dealt round-robin to 8 XCDs)
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  tile_body<Real, RB>(d, tile, in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x,
                      true);
}

// The common pass shape with its structure fixed at compile time: two
// register groups, the first full (RB stages, per-thread factors of the
// lower pass bits), the last with NSTL stages (it holds pass bit 0, so it
// has no such factors), and (EXT) the diagonal of the controls below the
// pass.  With nothing left to decide at run time that changes the data
// registers, no path merges are needed: the generic kernel spends about a
// third of its vector instructions on register moves that reconcile its
// run-time branches.
//
// W4: the four-wave form for 512-thread workgroups of 2^14 complex64
// elements (two workgroups per CU at 128 VGPRs per lane): the reads of the
// below-pass diagonal's table entries are issued after the exchange and the
// factors are applied in two steps, so that fewer registers are live.
template <typename Real, int RB, int NSTL, bool EXT, bool NT, bool W4 = false>
__device__ __forceinline__ void pass2_tile(const PassDesc &d, uint32_t tile, const cplx<Real> *in,
                                           cplx<Real> *out, cplx<Real> *lds, uint32_t tid) {
  using C = cplx<Real>;
  constexpr int R = 1 << RB;
  const int TR = d.T - RB;
  const uint32_t base = tile_base(d, tile);
  const uint32_t st_thr = deposit_tid(tid, d.st_thr_w, TR);

  // every table read first: they are in flight together with the tile's.
  // The first group's factors come from the planner's per-thread table
  // (the same table entries, 64 consecutive ones per wave).
  C gf[RB];
  {
    const C *__restrict__ gt = (const C *)d.gtab;
#pragma unroll
    for (int q = 0; q < RB; ++q) gf[q] = gt[(uint32_t)q * blockDim.x + tid];
  }
  ExtRaw<Real, RB> raw;
  if (EXT && !W4) ext_loads<Real, RB>(d, base | st_thr, raw);

  C v[R];
  {
    const C *src = in + (base | deposit_tid(tid, d.ld_thr_w, TR));
#pragma unroll
    for (int rho = 0; rho < R; ++rho) v[rho] = ld_elem<NT>(src + deposit_reg<RB>(rho, d.ld_reg_w));
  }
  conj_if<RB>(v, d.conj_in != 0);
  if (d.norm_part) norm_partial<Real, RB>(v, d.norm_part, tile, tid);

  // (four-wave form: scheduling fences around the first network keep the
  // loads, the network and the factors from being interleaved into a
  // register peak above the 128-VGPR budget)
  if constexpr (W4) __builtin_amdgcn_sched_barrier(0);
  radix_network<Real, RB>(v, RB);
  if constexpr (W4) __builtin_amdgcn_sched_barrier(0);
  apply_factors_k<Real, RB, W4>(v, gf, C{(Real)1, (Real)0}, false);
  // (four-wave form: keep the exchange's LDS addresses from being computed
  // early, where they would be live across the network and spill)
  if constexpr (W4) __builtin_amdgcn_sched_barrier(0);
  if constexpr (sizeof(Real) == 4 || W4) {
    exchange_split<Real, RB, W4>(v, lds, d.grp[0], d.grp[1], tid, TR);  // half-tile LDS
  } else {
    exchange<Real, RB>(v, lds, d.grp[0], d.grp[1], tid, TR, true);
  }
  if (EXT && W4) ext_loads<Real, RB>(d, base | st_thr, raw);
  radix_network<Real, RB>(v, NSTL);

  if (EXT) {
    C f[RB], f0;
    ext_finish<Real, RB>(d, raw, f, f0);
    apply_factors_k<Real, RB, W4>(v, f, f0, true);
  } else {
    const Real scale = (Real)d.scale;
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
      v[rho].x *= scale;
      v[rho].y *= scale;
    }
  }
  conj_if<RB>(v, d.conj_out != 0);
  const uint32_t obase = d.reverse ? rev_bits(base, d.n) : base;
  store_tile_raw<Real, RB, NT>(d, v, out + (obase | st_thr));
}

template <typename Real, int RB, int NSTL, bool EXT, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? (RB >= 5 ? 256 : RB >= 3 ? 512 : 1024)
                                                   : (RB >= 5 ? 512 : 1024))
k_fused_pass2(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  pass2_tile<Real, RB, NSTL, EXT, NT>(d, tile, in, out,
                                      reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

// Cross-lane exchange of register bit q with lane bit LB of one 32-bit
// component, between the register pair (a: register bit q clear, b: set).
// Afterwards register bit q carries what lane bit LB carried and lane bit LB
// what register bit q carried: a lane whose bit LB is clear keeps a and takes
// its partner's a into b; a lane whose bit LB is set keeps b and takes its
// partner's b into a (partner = lane ^ 2^LB).
template <int LB>
__device__ __forceinline__ void lane_swap_u32(uint32_t &a, uint32_t &b, uint32_t lane) {
  if constexpr (LB == 5) {
    // v_permlane32_swap: the upper 32 lanes of a trade places with the lower
    // 32 lanes of b
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else if constexpr (LB == 4) {
    // v_permlane16_swap: the odd 16-lane rows of a trade places with the
    // even rows of b
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    static_assert(LB == 3, "lane bits 3..5 only");
    // rotating a 16-lane row by 8 (DPP row_ror:8) pairs lane l with l ^ 8
    const bool up = (lane >> 3) & 1u;
    const uint32_t send = up ? a : b;
    const uint32_t recv = (uint32_t)__builtin_amdgcn_mov_dpp((int)send, 0x128, 0xf, 0xf, false);
    if (up) a = recv;
    else b = recv;
  }
}

template <int LB>
__device__ __forceinline__ void lane_swap(cplx<float> &a, cplx<float> &b, uint32_t lane) {
  uint32_t ax = __float_as_uint(a.x), bx = __float_as_uint(b.x);
  uint32_t ay = __float_as_uint(a.y), by = __float_as_uint(b.y);
  lane_swap_u32<LB>(ax, bx, lane);
  lane_swap_u32<LB>(ay, by, lane);
  a = cplx<float>{__uint_as_float(ax), __uint_as_float(ay)};
  b = cplx<float>{__uint_as_float(bx), __uint_as_float(by)};
}

template <int LB>
__device__ __forceinline__ void lane_swap(cplx<double> &a, cplx<double> &b, uint32_t lane) {
  uint64_t w[4] = {(uint64_t)__double_as_longlong(a.x), (uint64_t)__double_as_longlong(a.y),
                   (uint64_t)__double_as_longlong(b.x), (uint64_t)__double_as_longlong(b.y)};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    uint32_t alo = (uint32_t)w[c], ahi = (uint32_t)(w[c] >> 32);
    uint32_t blo = (uint32_t)w[c + 2], bhi = (uint32_t)(w[c + 2] >> 32);
    lane_swap_u32<LB>(alo, blo, lane);
    lane_swap_u32<LB>(ahi, bhi, lane);
    w[c] = ((uint64_t)ahi << 32) | alo;
    w[c + 2] = ((uint64_t)bhi << 32) | blo;
  }
  a = cplx<double>{__longlong_as_double((long long)w[0]), __longlong_as_double((long long)w[1])};
  b = cplx<double>{__longlong_as_double((long long)w[2]), __longlong_as_double((long long)w[3])};
}

// Register bits 0..S-1 trade places with lane bits 5, 4, 3 (register bit q
// with lane bit 5 - q): the last group of a three-group pass takes the pass
// bits that the middle group held on those lanes.
template <typename Real, int RB, int S>
__device__ __forceinline__ void lane_swaps(cplx<Real> (&v)[1 << RB], uint32_t lane) {
#pragma unroll
  for (int q = 0; q < S; ++q) {
#pragma unroll
    for (int rho = 0; rho < (1 << RB); ++rho) {
      if (rho & (1 << q)) continue;
      if (q == 0) lane_swap<5>(v[rho], v[rho | 1], lane);
      else if (q == 1) lane_swap<4>(v[rho], v[rho | 2], lane);
      else lane_swap<3>(v[rho], v[rho | 4], lane);
    }
  }
}

// A pass of 10 + S bits with its structure fixed at compile time: groups 0
// and 1 full (RB stages each, per-thread factors of the lower pass bits from
// the planner's tables), one LDS exchange between them, then the S lowest
// pass bits brought into registers by cross-lane swaps (they sit on lane
// bits 5, 4, 3 of group 1's thread map) and applied by a radix-2^S network,
// and (EXT) the diagonal of the controls below the pass.  Wider middle
// passes let the first and last passes keep long contiguous rows.
// W4 as for pass2_tile.
template <typename Real, int RB, int S, bool EXT, bool NT, bool W4 = false>
__device__ __forceinline__ void pass3_tile(const PassDesc &d, uint32_t tile, const cplx<Real> *in,
                                           cplx<Real> *out, cplx<Real> *lds, uint32_t tid) {
  using C = cplx<Real>;
  constexpr int R = 1 << RB;
  const int TR = d.T - RB;
  const uint32_t base = tile_base(d, tile);
  const uint32_t st_thr = deposit_tid(tid, d.st_thr_w, TR);

  C gf[RB];
  {
    const C *__restrict__ gt = (const C *)d.gtab;
#pragma unroll
    for (int q = 0; q < RB; ++q) gf[q] = gt[(uint32_t)q * blockDim.x + tid];
  }
  ExtRaw<Real, RB> raw;
  if (EXT && !W4) ext_loads<Real, RB>(d, base | st_thr, raw);

  C v[R];
  {
    const C *src = in + (base | deposit_tid(tid, d.ld_thr_w, TR));
#pragma unroll
    for (int rho = 0; rho < R; ++rho) v[rho] = ld_elem<NT>(src + deposit_reg<RB>(rho, d.ld_reg_w));
  }
  conj_if<RB>(v, d.conj_in != 0);
  if (d.norm_part) norm_partial<Real, RB>(v, d.norm_part, tile, tid);

  // (four-wave form: scheduling fences around the first network keep the
  // loads, the network and the factors from being interleaved into a
  // register peak above the 128-VGPR budget)
  if constexpr (W4) __builtin_amdgcn_sched_barrier(0);
  radix_network<Real, RB>(v, RB);
  if constexpr (W4) __builtin_amdgcn_sched_barrier(0);
  apply_factors_k<Real, RB, W4>(v, gf, C{(Real)1, (Real)0}, false);
  {
    // group 1's factors: their reads are in flight during the exchange
    const C *__restrict__ gt = (const C *)d.gtab1;
#pragma unroll
    for (int q = 0; q < RB; ++q) gf[q] = gt[(uint32_t)q * blockDim.x + tid];
  }
  if constexpr (W4) __builtin_amdgcn_sched_barrier(0);  // as in pass2_tile
  if constexpr (sizeof(Real) == 4 || W4) {
    exchange_split<Real, RB, W4>(v, lds, d.grp[0], d.grp[1], tid, TR);  // half-tile LDS
  } else {
    exchange<Real, RB>(v, lds, d.grp[0], d.grp[1], tid, TR, true);
  }
  if (EXT && W4) ext_loads<Real, RB>(d, base | st_thr, raw);
  radix_network<Real, RB>(v, RB);
  apply_factors_k<Real, RB, W4>(v, gf, C{(Real)1, (Real)0}, false);
  lane_swaps<Real, RB, S>(v, tid & 63u);
  radix_network<Real, RB>(v, S);

  if (EXT) {
    C f[RB], f0;
    ext_finish<Real, RB>(d, raw, f, f0);
    apply_factors_k<Real, RB, W4>(v, f, f0, true);
  } else {
    const Real scale = (Real)d.scale;
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
      v[rho].x *= scale;
      v[rho].y *= scale;
    }
  }
  conj_if<RB>(v, d.conj_out != 0);
  const uint32_t obase = d.reverse ? rev_bits(base, d.n) : base;
  store_tile_raw<Real, RB, NT>(d, v, out + (obase | st_thr));
}

template <typename Real, int S, bool EXT, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_fused_pass3(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  pass3_tile<Real, 5, S, EXT, NT>(d, tile, in, out, reinterpret_cast<cplx<Real> *>(qft_smem),
                                  threadIdx.x);
}

// The lean (four-wave) forms of the compile-time kernels, for 512-thread
// complex64 workgroups of 2^14-element tiles: the W4 code path (table reads
// of the below-pass diagonal after the exchange, two-step factors,
// scheduling fences) at 128 VGPRs, four waves per SIMD, two workgroups per
// CU.  (The same path for complex128 at 256 VGPRs, two waves per SIMD
// instead of one, measured slower: 5.98 against 5.50 ms at n = 28, the
// late table reads costing more than the second workgroup gains.)
#define QFT_LEAN_BOUNDS(Real) \
  __launch_bounds__(sizeof(Real) == 4 ? 512 : 256)                                            \
      __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 4 : 2)))

template <typename Real, int RB, int NSTL, bool EXT, bool NT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_fused_pass2w(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  pass2_tile<Real, RB, NSTL, EXT, NT, true>(d, tile, in, out,
                                           reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int S, bool EXT, bool NT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_fused_pass3w(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  pass3_tile<Real, 5, S, EXT, NT, true>(d, tile, in, out,
                                        reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

// The lean form runs every complex64 compile-time pass of 512 threads
// (2^14-element tiles) and every complex128 one of 256 threads (2^13).
inline bool lean_form(const PassLaunch &L, bool c128) { return L.threads == (c128 ? 256 : 512); }
inline bool lean_group(const BatchGroup &g, bool c128) { return g.threads == (c128 ? 256 : 512); }

int fused_pass_shape(const PassLaunch &L) { return pass_kernel_shape(L); }

template <typename Real, int RB>
static hipError_t launch_pass_t(const PassLaunch &L, const void *in, void *out, hipStream_t s) {
  auto fn = k_fused_pass<Real, RB>;
  if constexpr (RB == 5) {
    const int shape = fused_pass_shape(L);
    if (shape > 10) {
      using K = void (*)(const PassDesc, const cplx<Real> *, cplx<Real> *);
#define QFT_P3(E, N) \
  {k_fused_pass3<Real, 1, E, N>, k_fused_pass3<Real, 2, E, N>, k_fused_pass3<Real, 3, E, N>}
      static const K tab3[2][2][3] = {{QFT_P3(false, false), QFT_P3(true, false)},
                                      {QFT_P3(false, true), QFT_P3(true, true)}};
#undef QFT_P3
      fn = tab3[L.d.nt ? 1 : 0][L.d.ext_tw ? 1 : 0][L.d.lane_swap - 1];
      {
        if (lean_form(L, sizeof(Real) == 8)) {
#define QFT_P3W(E, N) \
  {k_fused_pass3w<Real, 1, E, N>, k_fused_pass3w<Real, 2, E, N>, k_fused_pass3w<Real, 3, E, N>}
          static const K tab3w[2][2][3] = {{QFT_P3W(false, false), QFT_P3W(true, false)},
                                           {QFT_P3W(false, true), QFT_P3W(true, true)}};
#undef QFT_P3W
          fn = tab3w[L.d.nt ? 1 : 0][L.d.ext_tw ? 1 : 0][L.d.lane_swap - 1];
        }
      }
    } else if (shape) {
      using K = void (*)(const PassDesc, const cplx<Real> *, cplx<Real> *);
#define QFT_P2(E, N)                                                                         \
  {k_fused_pass2<Real, 5, 1, E, N>, k_fused_pass2<Real, 5, 2, E, N>,                        \
   k_fused_pass2<Real, 5, 3, E, N>, k_fused_pass2<Real, 5, 4, E, N>,                        \
   k_fused_pass2<Real, 5, 5, E, N>}
      static const K tab[2][2][5] = {{QFT_P2(false, false), QFT_P2(true, false)},
                                     {QFT_P2(false, true), QFT_P2(true, true)}};
#undef QFT_P2
      fn = tab[L.d.nt ? 1 : 0][L.d.ext_tw ? 1 : 0][L.d.grp[1].nst - 1];
      {
        if (lean_form(L, sizeof(Real) == 8)) {
#define QFT_P2W(E, N)                                                                        \
  {k_fused_pass2w<Real, 5, 1, E, N>, k_fused_pass2w<Real, 5, 2, E, N>,                       \
   k_fused_pass2w<Real, 5, 3, E, N>, k_fused_pass2w<Real, 5, 4, E, N>,                       \
   k_fused_pass2w<Real, 5, 5, E, N>}
          static const K tabw[2][2][5] = {{QFT_P2W(false, false), QFT_P2W(true, false)},
                                          {QFT_P2W(false, true), QFT_P2W(true, true)}};
#undef QFT_P2W
          fn = tabw[L.d.nt ? 1 : 0][L.d.ext_tw ? 1 : 0][L.d.grp[1].nst - 1];
        }
      }
    }
  }
  if (L.lds_bytes > 65536) {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void *>(fn), 163840);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(L.grid), dim3(L.threads), L.lds_bytes, s, L.d,
                     (const cplx<Real> *)in, (cplx<Real> *)out);
  return hipGetLastError();
}

hipError_t launch_fused_pass(const PassLaunch &L, bool c128, const void *in, void *out,
                             hipStream_t s) {
  const int r = L.d.r;
  if (c128) {
    switch (r) {
      case 1: return launch_pass_t<double, 1>(L, in, out, s);
      case 2: return launch_pass_t<double, 2>(L, in, out, s);
      case 3: return launch_pass_t<double, 3>(L, in, out, s);
      case 4: return launch_pass_t<double, 4>(L, in, out, s);
      case 5: return launch_pass_t<double, 5>(L, in, out, s);
    }
  } else {
    switch (r) {
      case 1: return launch_pass_t<float, 1>(L, in, out, s);
      case 2: return launch_pass_t<float, 2>(L, in, out, s);
      case 3: return launch_pass_t<float, 3>(L, in, out, s);
      case 4: return launch_pass_t<float, 4>(L, in, out, s);
      case 5: return launch_pass_t<float, 5>(L, in, out, s);
    }
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// batched launches
// ---------------------------------------------------------------------------

// One launch of a batch group: the tiles of many transforms that share a pass
// level, a register radix and a workgroup size, one tile per workgroup.
// Workgroup b finds its segment (transform pass) by binary search over the
// segments' first items.  Passes of one transform are in different launches,
// ordered on the stream, so no workgroup ever waits for another.
template <typename Real, int RB>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? (RB >= 5 ? 256 : RB >= 3 ? 512 : 1024)
                                                   : (RB >= 5 ? 512 : 1024))
k_batch_group(const BatchSeg *__restrict__ segs, int nseg, const PassDesc *__restrict__ descs,
              const BatchIO *__restrict__ io) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t item = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  const BatchSeg sg = segs[lo];
  const BatchIO b = io[sg.desc];
  tile_body<Real, RB>(descs[sg.desc], item - sg.first, (const cplx<Real> *)b.in,
                      (cplx<Real> *)b.out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x,
                      true);
}

// The same for groups whose passes all have the two-group shape (see
// k_fused_pass2), so that a transform gives bit-identical results alone and
// in a batch.
template <typename Real, int NSTL, bool EXT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_batch_group2(const BatchSeg *__restrict__ segs, int nseg, const PassDesc *__restrict__ descs,
               const BatchIO *__restrict__ io) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t item = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  const BatchSeg sg = segs[lo];
  const BatchIO b = io[sg.desc];
  pass2_tile<Real, 5, NSTL, EXT, false>(descs[sg.desc], item - sg.first, (const cplx<Real> *)b.in,
                                 (cplx<Real> *)b.out, reinterpret_cast<cplx<Real> *>(qft_smem),
                                 threadIdx.x);
}

// The same for groups of three-group passes.
template <typename Real, int S, bool EXT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_batch_group3(const BatchSeg *__restrict__ segs, int nseg, const PassDesc *__restrict__ descs,
               const BatchIO *__restrict__ io) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t item = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  const BatchSeg sg = segs[lo];
  const BatchIO b = io[sg.desc];
  pass3_tile<Real, 5, S, EXT, false>(descs[sg.desc], item - sg.first, (const cplx<Real> *)b.in,
                                     (cplx<Real> *)b.out, reinterpret_cast<cplx<Real> *>(qft_smem),
                                     threadIdx.x);
}

// Lean batch forms (see k_fused_pass2w), so that a transform gives
// bit-identical results alone and in a batch.
template <typename Real, int NSTL, bool EXT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_batch_group2w(const BatchSeg *__restrict__ segs, int nseg, const PassDesc *__restrict__ descs,
                const BatchIO *__restrict__ io) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t item = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  const BatchSeg sg = segs[lo];
  const BatchIO b = io[sg.desc];
  pass2_tile<Real, 5, NSTL, EXT, false, true>(descs[sg.desc], item - sg.first,
                                              (const cplx<Real> *)b.in, (cplx<Real> *)b.out,
                                              reinterpret_cast<cplx<Real> *>(qft_smem),
                                              threadIdx.x);
}

template <typename Real, int S, bool EXT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_batch_group3w(const BatchSeg *__restrict__ segs, int nseg, const PassDesc *__restrict__ descs,
                const BatchIO *__restrict__ io) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t item = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  const BatchSeg sg = segs[lo];
  const BatchIO b = io[sg.desc];
  pass3_tile<Real, 5, S, EXT, false, true>(descs[sg.desc], item - sg.first,
                                           (const cplx<Real> *)b.in, (cplx<Real> *)b.out,
                                           reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int RB>
static hipError_t launch_group_t(const BatchGroup &g, hipStream_t s) {
  auto fn = k_batch_group<Real, RB>;
  if constexpr (RB == 5) {
    if (g.shape > 10) {
      using K = void (*)(const BatchSeg *, int, const PassDesc *, const BatchIO *);
      static const K tab3[6] = {k_batch_group3<Real, 1, false>, k_batch_group3<Real, 2, false>,
                                k_batch_group3<Real, 3, false>, k_batch_group3<Real, 1, true>,
                                k_batch_group3<Real, 2, true>,  k_batch_group3<Real, 3, true>};
      fn = tab3[g.shape - 11];
      {
        if (lean_group(g, sizeof(Real) == 8)) {
          static const K tab3w[6] = {
              k_batch_group3w<Real, 1, false>, k_batch_group3w<Real, 2, false>,
              k_batch_group3w<Real, 3, false>, k_batch_group3w<Real, 1, true>,
              k_batch_group3w<Real, 2, true>,  k_batch_group3w<Real, 3, true>};
          fn = tab3w[g.shape - 11];
        }
      }
    } else if (g.shape) {
      using K = void (*)(const BatchSeg *, int, const PassDesc *, const BatchIO *);
      static const K tab[10] = {
          k_batch_group2<Real, 1, false>, k_batch_group2<Real, 2, false>,
          k_batch_group2<Real, 3, false>, k_batch_group2<Real, 4, false>,
          k_batch_group2<Real, 5, false>, k_batch_group2<Real, 1, true>,
          k_batch_group2<Real, 2, true>,  k_batch_group2<Real, 3, true>,
          k_batch_group2<Real, 4, true>,  k_batch_group2<Real, 5, true>};
      fn = tab[g.shape - 1];
      {
        if (lean_group(g, sizeof(Real) == 8)) {
          static const K tabw[10] = {
              k_batch_group2w<Real, 1, false>, k_batch_group2w<Real, 2, false>,
              k_batch_group2w<Real, 3, false>, k_batch_group2w<Real, 4, false>,
              k_batch_group2w<Real, 5, false>, k_batch_group2w<Real, 1, true>,
              k_batch_group2w<Real, 2, true>,  k_batch_group2w<Real, 3, true>,
              k_batch_group2w<Real, 4, true>,  k_batch_group2w<Real, 5, true>};
          fn = tabw[g.shape - 1];
        }
      }
    }
  }
  if (g.lds_bytes > 65536) {
    hipError_t e = ensure_lds_limit(reinterpret_cast<const void *>(fn), 163840);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(g.items), dim3(g.threads), g.lds_bytes, s, g.segs, g.nseg, g.descs,
                     g.io);
  return hipGetLastError();
}

hipError_t launch_batch_group(bool c128, const BatchGroup &g, hipStream_t s) {
  if (c128) {
    switch (g.r) {
      case 1: return launch_group_t<double, 1>(g, s);
      case 2: return launch_group_t<double, 2>(g, s);
      case 3: return launch_group_t<double, 3>(g, s);
      case 4: return launch_group_t<double, 4>(g, s);
      case 5: return launch_group_t<double, 5>(g, s);
    }
  } else {
    switch (g.r) {
      case 1: return launch_group_t<float, 1>(g, s);
      case 2: return launch_group_t<float, 2>(g, s);
      case 3: return launch_group_t<float, 3>(g, s);
      case 4: return launch_group_t<float, 4>(g, s);
      case 5: return launch_group_t<float, 5>(g, s);
    }
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// gate-by-gate sweeps
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t insert_bit(uint32_t x, int pos, uint32_t bit) {
  const uint32_t lowmask = (1u << pos) - 1u;
  return ((x & ~lowmask) << 1) | (bit << pos) | (x & lowmask);
}

template <typename Real>
__global__ void k_h(cplx<Real> *psi, int t, uint32_t npairs, Real s) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < npairs;
       i += gridDim.x * blockDim.x) {
    const uint32_t i0 = insert_bit(i, t, 0u);
    const uint32_t i1 = i0 | (1u << t);
    const cplx<Real> a = psi[i0], b = psi[i1];
    psi[i0] = {(a.x + b.x) * s, (a.y + b.y) * s};
    psi[i1] = {(a.x - b.x) * s, (a.y - b.y) * s};
  }
}

// controlled phase: multiply amplitudes with bits c and t set (c < t)
template <typename Real>
__global__ void k_cphase(cplx<Real> *psi, int c, int t, uint32_t nquads, cplx<Real> ph) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nquads;
       i += gridDim.x * blockDim.x) {
    const uint32_t idx = insert_bit(insert_bit(i, c, 1u), t, 1u);
    psi[idx] = cmul(psi[idx], ph);
  }
}

// swap qubits a < b: exchange the (bit a, bit b) = (1, 0) and (0, 1) amplitudes
template <typename Real>
__global__ void k_swap(cplx<Real> *psi, int a, int b, uint32_t nquads) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nquads;
       i += gridDim.x * blockDim.x) {
    const uint32_t base = insert_bit(insert_bit(i, a, 0u), b, 0u);
    const uint32_t i10 = base | (1u << a);
    const uint32_t i01 = base | (1u << b);
    const cplx<Real> x = psi[i10];
    psi[i10] = psi[i01];
    psi[i01] = x;
  }
}

template <typename Real>
__global__ void k_scale(cplx<Real> *psi, uint32_t N, Real f) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    psi[i].x *= f;
    psi[i].y *= f;
  }
}

static dim3 sweep_grid(uint32_t work) {
  uint32_t blocks = (work + 255u) / 256u;
  if (blocks > 65536u) blocks = 65536u;
  if (blocks == 0) blocks = 1;
  return dim3(blocks);
}

hipError_t launch_h(void *psi, int n, int t, bool c128, hipStream_t s) {
  const uint32_t work = 1u << (n - 1);
  if (c128)
    hipLaunchKernelGGL(k_h<double>, sweep_grid(work), dim3(256), 0, s, (cplx<double> *)psi, t,
                       work, 0.70710678118654752440);
  else
    hipLaunchKernelGGL(k_h<float>, sweep_grid(work), dim3(256), 0, s, (cplx<float> *)psi, t,
                       work, 0.70710678118654752440f);
  return hipGetLastError();
}

hipError_t launch_cphase(void *psi, int n, int c, int t, double re, double im, bool c128,
                         hipStream_t s) {
  const uint32_t work = 1u << (n - 2);
  if (c128)
    hipLaunchKernelGGL(k_cphase<double>, sweep_grid(work), dim3(256), 0, s, (cplx<double> *)psi,
                       c, t, work, cplx<double>{re, im});
  else
    hipLaunchKernelGGL(k_cphase<float>, sweep_grid(work), dim3(256), 0, s, (cplx<float> *)psi, c,
                       t, work, cplx<float>{(float)re, (float)im});
  return hipGetLastError();
}

hipError_t launch_swap(void *psi, int n, int a, int b, bool c128, hipStream_t s) {
  const uint32_t work = 1u << (n - 2);
  if (c128)
    hipLaunchKernelGGL(k_swap<double>, sweep_grid(work), dim3(256), 0, s, (cplx<double> *)psi, a,
                       b, work);
  else
    hipLaunchKernelGGL(k_swap<float>, sweep_grid(work), dim3(256), 0, s, (cplx<float> *)psi, a,
                       b, work);
  return hipGetLastError();
}

hipError_t launch_scale(void *psi, int n, double f, bool c128, hipStream_t s) {
  const uint32_t work = 1u << n;
  if (c128)
    hipLaunchKernelGGL(k_scale<double>, sweep_grid(work), dim3(256), 0, s, (cplx<double> *)psi,
                       work, f);
  else
    hipLaunchKernelGGL(k_scale<float>, sweep_grid(work), dim3(256), 0, s, (cplx<float> *)psi,
                       work, (float)f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// input norm ||x||_2 (the paper's scale_in, Sec. 3 step 1) as metadata
// ---------------------------------------------------------------------------

// Standalone partial sums of |x|^2 (used by the gate-by-gate schedule; the
// fused schedule folds them into its first pass): workgroup b sums a
// contiguous block in FP64 and writes part[b].
template <typename Real>
__global__ void __launch_bounds__(256) k_norm_sweep(const cplx<Real> *psi, uint32_t N,
                                                    double *part) {
  __shared__ double red[4];
  const uint32_t per = (N + gridDim.x - 1) / gridDim.x;
  const uint32_t lo = blockIdx.x * per;
  const uint32_t hi = lo + per < N ? lo + per : N;
  double a = 0.0;
  for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double x = (double)psi[i].x, y = (double)psi[i].y;
    a += x * x + y * y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[0] = sqrt(sum of part[0..count)), summed in a fixed order.
__global__ void __launch_bounds__(256) k_norm_finish(const double *part, uint32_t count,
                                                     double *out) {
  __shared__ double red[256];
  double a = 0.0;
  for (uint32_t i = threadIdx.x; i < count; i += 256) a += part[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

hipError_t launch_norm_sweep(const void *psi, int n, bool c128, double *part, uint32_t nparts,
                             hipStream_t s) {
  const uint32_t N = 1u << n;
  if (c128)
    hipLaunchKernelGGL(k_norm_sweep<double>, dim3(nparts), dim3(256), 0, s,
                       (const cplx<double> *)psi, N, part);
  else
    hipLaunchKernelGGL(k_norm_sweep<float>, dim3(nparts), dim3(256), 0, s,
                       (const cplx<float> *)psi, N, part);
  return hipGetLastError();
}

hipError_t launch_norm_finish(const double *part, uint32_t count, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(256), 0, s, part, count, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// zero padding to a power of two
// ---------------------------------------------------------------------------

template <typename Real>
__global__ void __launch_bounds__(256) k_pad(const cplx<Real> *src, uint64_t count,
                                             cplx<Real> *dst, uint64_t N) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = i < count ? src[i] : cplx<Real>{(Real)0, (Real)0};
}

hipError_t launch_pad(const void *src, size_t count, void *dst, int n, bool c128, hipStream_t s) {
  const uint64_t N = 1ull << n;
  const uint64_t blocks = (N + 255) / 256;
  const dim3 grid((unsigned)(blocks < 65536 ? blocks : 65536));
  if (c128)
    hipLaunchKernelGGL(k_pad<double>, grid, dim3(256), 0, s, (const cplx<double> *)src,
                       (uint64_t)count, (cplx<double> *)dst, N);
  else
    hipLaunchKernelGGL(k_pad<float>, grid, dim3(256), 0, s, (const cplx<float> *)src,
                       (uint64_t)count, (cplx<float> *)dst, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Philox-4x32-10 input generator
// ---------------------------------------------------------------------------

struct u32x4 {
  uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c.v[0];
    const uint64_t p1 = (uint64_t)M1 * c.v[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    u32x4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
  }
  return c;
}

template <typename Real>
__global__ void k_fill_random(cplx<Real> *psi, uint32_t N, int dist, uint64_t seed,
                              uint64_t stream_id) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    u32x4 c;
    c.v[0] = i;
    c.v[1] = 0u;
    c.v[2] = (uint32_t)stream_id;
    c.v[3] = (uint32_t)(stream_id >> 32);
    const u32x4 w = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double a = (double)((((uint64_t)w.v[1] << 32) | w.v[0]) >> 11);
    const double b = (double)((((uint64_t)w.v[3] << 32) | w.v[2]) >> 11);
    const double two53 = 1.1102230246251565404e-16;  // 2^-53
    double re, im;
    if (dist == 0) {
      const double u1 = (a + 0.5) * two53;
      const double u2 = (b + 0.5) * two53;
      const double r = sqrt(-2.0 * log(u1));
      const double th = 6.283185307179586232 * u2;
      re = r * cos(th);
      im = r * sin(th);
    } else {
      re = 2.0 * (a * two53) - 1.0;
      im = 2.0 * (b * two53) - 1.0;
    }
    psi[i] = {(Real)re, (Real)im};
  }
}

hipError_t launch_fill_random(void *psi, int n, bool c128, int dist, uint64_t seed,
                              uint64_t stream_id, hipStream_t s) {
  const uint32_t N = 1u << n;
  if (c128)
    hipLaunchKernelGGL(k_fill_random<double>, sweep_grid(N), dim3(256), 0, s,
                       (cplx<double> *)psi, N, dist, seed, stream_id);
  else
    hipLaunchKernelGGL(k_fill_random<float>, sweep_grid(N), dim3(256), 0, s, (cplx<float> *)psi,
                       N, dist, seed, stream_id);
  return hipGetLastError();
}

}  // namespace qft
