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

#include "qft_internal.h"
#include "qft_kernels.h"

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

// LDS address of tile element e: the low SW bits are XORed with a fold of the
// higher bits, a bijection that spreads power-of-two strides over the banks.
template <typename Real>
__device__ __forceinline__ uint32_t lds_swizzle(uint32_t e) {
  constexpr int SW = sizeof(Real) == 4 ? 4 : 3;
  const uint32_t h = (e >> SW) ^ (e >> (2 * SW)) ^ (e >> (3 * SW)) ^ (e >> (4 * SW));
  return e ^ (h & ((1u << SW) - 1u));
}

__device__ __forceinline__ uint32_t deposit_tid(uint32_t tid, const uint8_t *pos, int nb) {
  uint32_t e = 0;
  for (int b = 0; b < nb; ++b) e |= ((tid >> b) & 1u) << pos[b];
  return e;
}

template <int RB>
__device__ __forceinline__ uint32_t deposit_reg(int rho, const uint8_t *pos) {
  uint32_t o = 0;
#pragma unroll
  for (int q = 0; q < RB; ++q)
    if ((rho >> q) & 1) o |= 1u << pos[q];
  return o;
}

// Apply the stages (targets) of one register group.
// Register bit q holds local pass bit jbase + q.  The twiddle of target
// jl = jbase + q on element (thread, rho) is w_{2^{jl+1}}^{u}, u = local pass
// bits below jl with the bits below jl - k cleared (AQFT); u splits into the
// thread's bits below jbase and the register bits below q, so
//   w_{2^{jl+1}}^{u} = w_{2^{jl+1}}^{u_thr} * w_{2^{q+1}}^{rho mod 2^q}.
template <typename Real, int RB>
__device__ __forceinline__ void apply_stages(cplx<Real> (&v)[1 << RB], const PassDesc &d,
                                             const GroupMap &G, uint32_t e_thr) {
  using C = cplx<Real>;
  constexpr int R = 1 << RB;
  const int nst = G.nst;
  const int jbase = G.jbase;
  const C *__restrict__ W = (const C *)d.tw_int;
  const uint32_t u_thr = (e_thr >> d.pbase) & ((1u << jbase) - 1u);
  const int MI1 = d.MI - 1;
#pragma unroll
  for (int q = RB - 1; q >= 0; --q) {
    if (q < nst) {
      const int jl = jbase + q;
      int clear = d.aqft ? jl - d.k : 0;
      clear = clear < 0 ? 0 : clear;
      const uint32_t x_thr = clear >= jbase ? 0u : ((u_thr >> clear) << clear);
      const int rclear = clear > jbase ? clear - jbase : 0;
      C tw[R / 2];
      tw[0] = W[x_thr << (MI1 - jl)];
#pragma unroll
      for (int a = 1; a < (1 << q); ++a) {
        const uint32_t xr = ((uint32_t)a >> rclear) << rclear;
        tw[a] = cmul(tw[0], W[xr << (MI1 - q)]);
      }
#pragma unroll
      for (int rho = 0; rho < R; ++rho) {
        if (rho & (1 << q)) continue;
        const int hi = rho | (1 << q);
        const C a = v[rho];
        const C b = v[hi];
        v[rho] = cadd(a, b);
        v[hi] = cmul(csub(a, b), tw[rho & ((1 << q) - 1)]);
      }
    }
  }
}

template <typename Real, int RB>
__global__ void __launch_bounds__(RB >= 5 ? 512 : 1024)
k_fused_pass(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  using C = cplx<Real>;
  constexpr int R = 1 << RB;
  extern __shared__ __align__(16) unsigned char qft_smem[];
  C *lds = reinterpret_cast<C *>(qft_smem);
  const uint32_t tid = threadIdx.x;
  const int TR = d.T - RB;

  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    // consecutive tiles on one XCD (workgroups are dealt round-robin to 8 XCDs)
    const uint32_t per = d.ntiles >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  uint32_t base = 0;
  for (int b = 0; b < d.nfree; ++b) base |= ((tile >> b) & 1u) << d.free_pos[b];

  C v[R];
  {
    const uint32_t g = base | deposit_tid(tid, d.ld_thr_g, TR);
#pragma unroll
    for (int rho = 0; rho < R; ++rho) v[rho] = in[g | deposit_reg<RB>(rho, d.ld_reg_g)];
  }

  for (int gi = 0; gi < d.ngroups; ++gi) {
    const GroupMap &G = d.grp[gi];
    const uint32_t e_thr = deposit_tid(tid, G.thr_pos, TR);
    if (gi > 0) {
      const GroupMap &P = d.grp[gi - 1];
      const uint32_t e_prev = deposit_tid(tid, P.thr_pos, TR);
#pragma unroll
      for (int rho = 0; rho < R; ++rho)
        lds[lds_swizzle<Real>(e_prev | deposit_reg<RB>(rho, P.reg_pos))] = v[rho];
      __syncthreads();
#pragma unroll
      for (int rho = 0; rho < R; ++rho)
        v[rho] = lds[lds_swizzle<Real>(e_thr | deposit_reg<RB>(rho, G.reg_pos))];
      __syncthreads();
    }
    apply_stages<Real, RB>(v, d, G, e_thr);
  }

  const Real scale = (Real)d.scale;
  const uint32_t obase = d.reverse ? rev_bits(base, d.n) : base;
  const uint32_t g = obase | deposit_tid(tid, d.st_thr_g, TR);
  const uint32_t nmask = d.n >= 32 ? 0xffffffffu : ((1u << d.n) - 1u);
#pragma unroll
  for (int rho = 0; rho < R; ++rho) {
    const uint32_t idx = g | deposit_reg<RB>(rho, d.st_reg_g);
    C val = v[rho];
    if (d.ext_tw) {
      // diagonal of the controlled phases with controls below the pass:
      // w_N^E, E = sum over pass bits j set of trunc_{lo+j-k}(v) 2^{n-1-lo-j}
      const uint32_t vv = idx & ((1u << d.lo) - 1u);
      const uint32_t p = (idx >> d.lo) & ((1u << d.m) - 1u);
      uint32_t E;
      if (!d.aqft) {
        E = (vv * rev_bits(p, d.m)) << (d.n - d.lo - d.m);
      } else {
        E = 0;
        for (int j = 0; j < d.m; ++j) {
          if ((p >> j) & 1u) {
            const int s = d.lo + j - d.k;
            const uint32_t tv = s <= 0 ? vv : (s >= d.lo ? 0u : ((vv >> s) << s));
            E = (E + (tv << (d.n - 1 - d.lo - j))) & nmask;
          }
        }
      }
      const C *__restrict__ tlo = (const C *)d.tw_lo;
      const C *__restrict__ thi = (const C *)d.tw_hi;
      C w = cmul(tlo[E & ((1u << d.L) - 1u)], thi[E >> d.L]);
      w.x *= scale;
      w.y *= scale;
      val = cmul(val, w);
    } else {
      val.x *= scale;
      val.y *= scale;
    }
    out[idx] = val;
  }
}

template <typename Real, int RB>
static hipError_t launch_pass_t(const PassLaunch &L, const void *in, void *out, hipStream_t s) {
  auto fn = k_fused_pass<Real, RB>;
  if (L.lds_bytes > 65536) {
    static int set = 0;
    if (!set) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
      if (e != hipSuccess) return e;
      set = 1;
    }
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
