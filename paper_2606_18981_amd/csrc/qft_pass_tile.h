// Device code of one tile of a fused pass, shared by the translation units
// that instantiate pass kernels (the transform's own kernels, and the last
// pass that also compares its output with a reference).
//
// A workgroup owns one tile of 2^T elements (m pass bits + spectator bits,
// see qft_internal.h).  Each thread holds R = 2^RB elements in registers; the
// pass bits are applied RB at a time (radix-2^RB decimation-in-frequency in
// registers), with an LDS exchange between register groups.  Per target
// qubit t the work is the circuit's H(t) (Fig. 1) - here an unnormalised
// butterfly, the 1/sqrt(2) factors being folded into one per-pass scale -
// followed by the product of the controlled phases of target t whose control
// lies inside the pass (Sec. 2: that product is the FFT twiddle T~).
// Controlled phases whose control lies below the pass are applied as one
// diagonal at the end of the pass.  The last pass writes bit-reversed
// addresses when the final swaps are requested (Sec. 3 step 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qft_internal.h"

namespace qft {

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

// Comparison of the stored tile with a reference output: the accuracy
// metrics of a transform folded into its last pass, so that the output is
// not read back.  Per thread, in FP64 over its elements y (the values just
// stored) and r = ref at the same output index: the kCmpSlots sums and
// maxima of qft_internal.h.  The wave combines its lanes in a fixed
// butterfly, and lane 0 writes the wave's partial to
// d.cmp_part[tile * waves + wave]; a workgroup smaller than a wave writes
// one partial per thread, as norm_partial does.  store_compare_tile takes
// the place of the tile's store: `obase` is the output index of the
// thread's register-0 element.  Every thread of the workgroup calls it.
//
// The tile is stored and the reference read in chunks of 4 elements, each
// chunk's sums taken DEPTH chunks after its reads are issued; scheduling
// fences between the chunks keep the compiler from computing every address
// up front (the addresses of all elements, live at once beside the data
// registers, spill the four-wave kernels).
struct CmpPart {
  double d2, r2, y2, cr, ci, md2, mr2, mri;
};

// a <- the combination of a and b.  Every step is commutative (sums, maxima,
// the larger |r|^2 with the lower index on ties), so two lanes that combine
// each other's partials end up with the same bits.
__device__ __forceinline__ void cmp_combine(CmpPart &a, const CmpPart &b) {
  a.d2 += b.d2;
  a.r2 += b.r2;
  a.y2 += b.y2;
  a.cr += b.cr;
  a.ci += b.ci;
  a.md2 = fmax(a.md2, b.md2);
  if (b.mr2 > a.mr2 || (b.mr2 == a.mr2 && b.mri < a.mri)) {
    a.mr2 = b.mr2;
    a.mri = b.mri;
  }
}

__device__ __forceinline__ CmpPart cmp_shfl_xor(const CmpPart &p, int off) {
  CmpPart q;
  q.d2 = __shfl_xor(p.d2, off, 64);
  q.r2 = __shfl_xor(p.r2, off, 64);
  q.y2 = __shfl_xor(p.y2, off, 64);
  q.cr = __shfl_xor(p.cr, off, 64);
  q.ci = __shfl_xor(p.ci, off, 64);
  q.md2 = __shfl_xor(p.md2, off, 64);
  q.mr2 = __shfl_xor(p.mr2, off, 64);
  q.mri = __shfl_xor(p.mri, off, 64);
  return q;
}

// A thread's running sums while it compares its elements (the argmax index
// kept as an integer until the partial is written).
struct CmpAcc {
  double d2, r2, y2, cr, ci, md2, mr2;
  uint32_t mi;
};

template <typename Real>
__device__ __forceinline__ void cmp_accumulate(CmpAcc &p, cplx<Real> y, cplx<Real> r,
                                               uint32_t index) {
  const double yx = (double)y.x, yy = (double)y.y;
  const double rx = (double)r.x, ry = (double)r.y;
  const double dx = yx - rx, dy = yy - ry;
  const double d2 = dx * dx + dy * dy;
  const double r2 = rx * rx + ry * ry;
  p.d2 += d2;
  p.r2 += r2;
  // the other sums take each product straight into the accumulator
  p.y2 = fma(yy, yy, fma(yx, yx, p.y2));
  p.cr = fma(ry, yy, fma(rx, yx, p.cr));  // conj(r) * y
  p.ci = fma(-ry, yx, fma(rx, yy, p.ci));
  p.md2 = fmax(p.md2, d2);
  // branch-free: a branch here splits the block, and the compiler then
  // moves the other sums past it, keeping every chunk's operands live
  const bool take = (r2 > p.mr2) | ((r2 == p.mr2) & (index < p.mi));
  p.mr2 = take ? r2 : p.mr2;
  p.mi = take ? index : p.mi;
}

// Reads of the reference for the first PRE chunks of 4 elements, issued
// before the pass's last register stages so that their latency is spent on
// that work.  `obase`: output index of the thread's register-0 element.
template <typename Real, int RB, int PRE>
__device__ __forceinline__ void cmp_prefetch(const PassDesc &d, uint32_t obase,
                                             cplx<Real> (&rv)[1 << RB]) {
  constexpr int R = 1 << RB;
  constexpr int K = R < 4 ? R : 4;
  constexpr int NP = PRE < R / K ? PRE : R / K;
  const cplx<Real> *ref = (const cplx<Real> *)d.cmp_ref + obase;
#pragma unroll
  for (int rho = 0; rho < NP * K; ++rho)
    rv[rho] = ld_elem<true>(ref + deposit_reg<RB>(rho, d.st_reg_w));  // read once: streaming
}

// The tile's store with the comparison: chunk by chunk, store, issue the
// reference reads DEPTH chunks ahead (those cmp_prefetch has not issued),
// and take the chunk's sums.
template <typename Real, int RB, bool NT, int PRE, int DEPTH>
__device__ __forceinline__ void store_compare_tile(const PassDesc &d,
                                                   const cplx<Real> (&v)[1 << RB],
                                                   cplx<Real> (&rv)[1 << RB], cplx<Real> *out,
                                                   uint32_t obase, uint32_t tile, uint32_t tid) {
  constexpr int R = 1 << RB;
  constexpr int K = R < 4 ? R : 4;  // elements per chunk
  constexpr int NC = R / K;         // chunks
  cplx<Real> *dst = out + obase;
  const cplx<Real> *ref = (const cplx<Real> *)d.cmp_ref + obase;
  CmpAcc acc{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0xffffffffu};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int rho = c * K + j;
      st_elem<NT>(dst + deposit_reg<RB>(rho, d.st_reg_w), v[rho]);
    }
    if (c + DEPTH >= PRE && c + DEPTH < NC) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int rho = (c + DEPTH) * K + j;
        rv[rho] = ld_elem<true>(ref + deposit_reg<RB>(rho, d.st_reg_w));
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int rho = c * K + j;
      cmp_accumulate<Real>(acc, v[rho], rv[rho], obase | deposit_reg<RB>(rho, d.st_reg_w));
    }
  }
  CmpPart p{acc.d2, acc.r2, acc.y2, acc.cr, acc.ci, acc.md2, acc.mr2, (double)acc.mi};
  __builtin_amdgcn_sched_barrier(0);
  const uint32_t threads = blockDim.x;
  size_t slot;
  if (threads >= 64) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) cmp_combine(p, cmp_shfl_xor(p, off));
    if ((tid & 63u) != 0) return;
    slot = (size_t)tile * (threads >> 6) + (tid >> 6);
  } else {
    slot = (size_t)tile * threads + tid;
  }
  double *o = d.cmp_part + slot * kCmpSlots;
  o[0] = p.d2;
  o[1] = p.r2;
  o[2] = p.y2;
  o[3] = p.cr;
  o[4] = p.ci;
  o[5] = p.md2;
  o[6] = p.mr2;
  o[7] = p.mri;
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
// needs) only take part in the barriers.  CMP: also compare the stored tile
// with d.cmp_ref (store_compare_tile; every thread must be active).
template <typename Real, int RB, bool CMP = false>
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
  if constexpr (CMP) {
    if (d.conj_out) conj_regs<Real, RB>(v);
    C rv[R];
    cmp_prefetch<Real, RB, 2>(d, obase | st_thr, rv);
    store_compare_tile<Real, RB, false, 2, 2>(d, v, rv, out, obase | st_thr, tile, tid);
  } else {
    store_tile<Real, RB>(d, v, out + (obase | st_thr));
  }
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
// W4: the four-wave form (512-thread complex64 workgroups of 2^14 elements
// at 128 VGPRs per lane, 256-thread complex128 ones of 2^13): the reads of
// the below-pass diagonal's table entries are issued after the exchange and
// the factors are applied in two steps, so that fewer registers are live.
// CMP: also compare the stored tile with d.cmp_ref (store_compare_tile).
// OX: store through the exchange-only third group (pass2x_shape), through
// the full-tile LDS area.
template <typename Real, int RB, int NSTL, bool EXT, bool NT, bool W4 = false, bool CMP = false,
          bool OX = false>
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
  // (four-wave form: a uniform branch; the branch-free sign flip keeps the
  // compiler from starting the first network before every load is back and
  // spills the 128-VGPR budget)
  if constexpr (W4) {
    if (d.conj_in) conj_regs<Real, RB>(v);
  } else {
    conj_if<RB>(v, d.conj_in != 0);
  }
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
  if constexpr ((sizeof(Real) == 4 || W4) && !OX) {
    exchange_split<Real, RB, W4>(v, lds, d.grp[0], d.grp[1], tid, TR);  // half-tile LDS
  } else {
    exchange<Real, RB>(v, lds, d.grp[0], d.grp[1], tid, TR, true);
  }
  if (EXT && W4) ext_loads<Real, RB>(d, base | st_thr, raw);
  // (CMP: the reference reads of the comparison start here, their latency
  // spent on the remaining stages; complex64 two-wave forms issue them all)
  constexpr int kCmpPre = W4 ? 1 : (sizeof(Real) == 4 ? 8 : 2);
  C rv[R];
  if constexpr (CMP)
    cmp_prefetch<Real, RB, kCmpPre>(d, (d.reverse ? rev_bits(base, d.n) : base) | st_thr, rv);
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
  if constexpr (OX) exchange<Real, RB>(v, lds, d.grp[1], d.grp[2], tid, TR, true);
  const uint32_t obase = d.reverse ? rev_bits(base, d.n) : base;
  if constexpr (CMP)
    store_compare_tile<Real, RB, NT, kCmpPre, W4 ? 1 : 2>(d, v, rv, out, obase | st_thr, tile,
                                                          tid);
  else
    store_tile_raw<Real, RB, NT>(d, v, out + (obase | st_thr));
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
// W4 and CMP as for pass2_tile.
template <typename Real, int RB, int S, bool EXT, bool NT, bool W4 = false, bool CMP = false>
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
  // (four-wave form: a uniform branch; the branch-free sign flip keeps the
  // compiler from starting the first network before every load is back and
  // spills the 128-VGPR budget)
  if constexpr (W4) {
    if (d.conj_in) conj_regs<Real, RB>(v);
  } else {
    conj_if<RB>(v, d.conj_in != 0);
  }
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
  // (CMP: the reference reads of the comparison start here, their latency
  // spent on the remaining stages; complex64 two-wave forms issue them all)
  constexpr int kCmpPre = W4 ? 1 : (sizeof(Real) == 4 ? 8 : 2);
  C rv[R];
  if constexpr (CMP)
    cmp_prefetch<Real, RB, kCmpPre>(d, (d.reverse ? rev_bits(base, d.n) : base) | st_thr, rv);
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
  if constexpr (CMP)
    store_compare_tile<Real, RB, NT, kCmpPre, W4 ? 1 : 2>(d, v, rv, out, obase | st_thr, tile,
                                                          tid);
  else
    store_tile_raw<Real, RB, NT>(d, v, out + (obase | st_thr));
}

// Launch bounds of the lean (four-wave) forms of the compile-time kernels,
// which take the W4 code path (table reads of the below-pass diagonal after
// the exchange, two-step factors, scheduling fences, the exchange in
// halves): 512-thread complex64 workgroups of 2^14 elements at 128 VGPRs
// per lane (four waves per SIMD), and 256-thread complex128 workgroups of
// 2^13 elements at up to 256 (two waves per SIMD); either way two
// workgroups per CU.
#define QFT_LEAN_BOUNDS(Real) \
  __launch_bounds__(sizeof(Real) == 4 ? 512 : 256)                                            \
      __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 4 : 2)))

// Tile of this workgroup.  With xcd_remap, consecutive tiles run on one XCD
// (workgroups are dealt round-robin to the 8 XCDs); for the middle pass of a
// three-pass plan that order measured about 20 % faster.
__device__ __forceinline__ uint32_t pass_tile_index(const PassDesc &d) {
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  return tile;
}

}  // namespace qft
