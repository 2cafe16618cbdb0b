// gfx950 kernels of the QFT->FFT path.
//
// k_fused_pass, k_fused_pass2, k_fused_pass3 and their four-wave forms: one
//   HBM pass of the fused schedule, one tile per workgroup (the tile code is
//   in qft_pass_tile.h); k_batch_group*: the same tiles for many transforms
//   in one launch.
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
#include "qft_pass_tile.h"

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


template <typename Real, int RB>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? (RB >= 5 ? 256 : RB >= 3 ? 512 : 1024)
                                                   : (RB >= 5 ? 512 : 1024))
k_fused_pass(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t tile = pass_tile_index(d);
  tile_body<Real, RB>(d, tile, in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x,
                      true);
}

template <typename Real, int RB, int NSTL, bool EXT, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? (RB >= 5 ? 256 : RB >= 3 ? 512 : 1024)
                                                   : (RB >= 5 ? 512 : 1024))
k_fused_pass2(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t tile = pass_tile_index(d);
  pass2_tile<Real, RB, NSTL, EXT, NT>(d, tile, in, out,
                                      reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

// The last pass of a bit-reversed-order plan: the two-group shape, then the
// exchange-only group that puts the lowest output bits on the lanes.
template <typename Real, int NSTL, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_fused_pass2x(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t tile = pass_tile_index(d);
  pass2_tile<Real, 5, NSTL, false, NT, false, false, true>(
      d, tile, in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int S, bool EXT, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_fused_pass3(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t tile = pass_tile_index(d);
  pass3_tile<Real, 5, S, EXT, NT>(d, tile, in, out, reinterpret_cast<cplx<Real> *>(qft_smem),
                                  threadIdx.x);
}

template <typename Real, int RB, int NSTL, bool EXT, bool NT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_fused_pass2w(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t tile = pass_tile_index(d);
  pass2_tile<Real, RB, NSTL, EXT, NT, true>(d, tile, in, out,
                                           reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int S, bool EXT, bool NT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_fused_pass3w(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  const uint32_t tile = pass_tile_index(d);
  pass3_tile<Real, 5, S, EXT, NT, true>(d, tile, in, out,
                                        reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

// Batch groups take the lean form on the same rule as lean_form.
inline bool lean_group(const BatchGroup &g, bool c128) { return g.threads == (c128 ? 256 : 512); }

int fused_pass_shape(const PassLaunch &L) { return pass_kernel_shape(L); }

template <typename Real, int RB>
static hipError_t launch_pass_t(const PassLaunch &L, const void *in, void *out, hipStream_t s) {
  auto fn = k_fused_pass<Real, RB>;
  if constexpr (RB == 5) {
    const int shape = fused_pass_shape(L);
    if (shape > 16) {
      using K = void (*)(const PassDesc, const cplx<Real> *, cplx<Real> *);
#define QFT_P2X(N)                                                                          \
  {k_fused_pass2x<Real, 1, N>, k_fused_pass2x<Real, 2, N>, k_fused_pass2x<Real, 3, N>,      \
   k_fused_pass2x<Real, 4, N>, k_fused_pass2x<Real, 5, N>}
      static const K tabx[2][5] = {QFT_P2X(false), QFT_P2X(true)};
#undef QFT_P2X
      fn = tabx[L.d.nt ? 1 : 0][shape - 17];
    } else if (shape > 10) {
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
    if (g.shape > 16) {
      // the store-exchange shape: the generic kernel (its tile's full LDS
      // area is what the plan allots)
    } else if (g.shape > 10) {
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
