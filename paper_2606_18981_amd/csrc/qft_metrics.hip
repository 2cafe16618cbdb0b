// Accuracy metrics of a transform against a reference on the device, and the
// closed-form expected error of the range-k AQFT; see include/qft_metrics.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>

#include "../../include/qft_metrics.h"
#include "qft_kernels.h"
#include "qft_pass_tile.h"
#include "qft_runtime.h"

using namespace qft;

namespace {

constexpr int kThreads = 256;
constexpr int kMaxExpectedBits = 20;  // closed form costs 2^M * M terms
constexpr int kMaxCombined = 1024;    // partials left for the finishing workgroup

__device__ __forceinline__ CmpPart cmp_load(const double *o) {
  return CmpPart{o[0], o[1], o[2], o[3], o[4], o[5], o[6], o[7]};
}

__device__ __forceinline__ void cmp_store(double *o, const CmpPart &a) {
  o[0] = a.d2;
  o[1] = a.r2;
  o[2] = a.y2;
  o[3] = a.cr;
  o[4] = a.ci;
  o[5] = a.md2;
  o[6] = a.mr2;
  o[7] = a.mri;
}

// Combine a workgroup's per-thread partials into one, written to out by
// thread 0: lanes in a fixed butterfly, then the waves in order, so that
// the result does not depend on scheduling.
__device__ __forceinline__ void cmp_reduce_block(CmpPart p, double *out) {
  __shared__ CmpPart red[kThreads / 64];
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) cmp_combine(p, cmp_shfl_xor(p, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = p;
  __syncthreads();
  if (threadIdx.x == 0) {
    CmpPart a = red[0];
    for (int w = 1; w < kThreads / 64; ++w) cmp_combine(a, red[w]);
    cmp_store(out, a);
  }
}

// Workgroup b reduces the contiguous block [b * per, min(N, (b + 1) * per))
// of y and r and writes its partial to part[b].  Each thread sums its
// elements in index order, with the per-element terms of the comparison
// folded into a transform's last pass (cmp_accumulate).
template <typename Real>
__global__ void __launch_bounds__(kThreads) k_compare_part(const cplx<Real> *y,
                                                           const cplx<Real> *r, uint64_t N,
                                                           uint64_t per, double *part) {
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < N ? lo + per : N;
  CmpAcc acc{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0xffffffffu};
  constexpr int U = 4;  // elements in flight per thread
  uint64_t i = lo + threadIdx.x;
  for (; i + (U - 1) * kThreads < hi; i += U * kThreads) {
    cplx<Real> ya[U], ra[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ya[u] = ld_elem<true>(y + i + u * kThreads);  // read once: streaming
      ra[u] = ld_elem<true>(r + i + u * kThreads);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) cmp_accumulate<Real>(acc, ya[u], ra[u], (uint32_t)(i + u * kThreads));
  }
  for (; i < hi; i += kThreads) cmp_accumulate<Real>(acc, y[i], r[i], (uint32_t)i);
  const CmpPart p{acc.d2, acc.r2, acc.y2, acc.cr, acc.ci, acc.md2, acc.mr2, (double)acc.mi};
  cmp_reduce_block(p, part + (size_t)blockIdx.x * kCmpSlots);
}

// Workgroup b combines the partials [b * per, min(count, (b + 1) * per)) of
// a compare pass into out[b] (each thread in index order, then the block).
__global__ void __launch_bounds__(kThreads) k_compare_combine(const double *part, uint64_t count,
                                                              uint64_t per, double *out) {
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < count ? lo + per : count;
  CmpPart p{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0.0};
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads)
    cmp_combine(p, cmp_load(part + i * kCmpSlots));
  cmp_reduce_block(p, out + (size_t)blockIdx.x * kCmpSlots);
}

// One workgroup: combine the partials in order, then form the metrics (the
// leakage reads y at the reference's argmax).
template <typename Real>
__global__ void __launch_bounds__(kThreads) k_compare_finish(const cplx<Real> *y, uint64_t N,
                                                             const double *part, int nparts,
                                                             double *out) {
  __shared__ CmpPart red[kThreads];
  CmpPart p{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kThreads)
    cmp_combine(p, cmp_load(part + (size_t)b * kCmpSlots));
  red[threadIdx.x] = p;
  __syncthreads();
  if (threadIdx.x == 0) {
    CmpPart a = red[0];
    for (int t = 1; t < kThreads; ++t) cmp_combine(a, red[t]);
    const double dn = sqrt(a.d2), rn = sqrt(a.r2), yn = sqrt(a.y2);
    const double rms = rn / sqrt((double)(N > 0 ? N : 1));
    const double md = sqrt(a.md2 > 0.0 ? a.md2 : 0.0);
    const uint64_t ks = (uint64_t)a.mri;
    const double yk2 = N > 0 ? (double)y[ks].x * (double)y[ks].x + (double)y[ks].y * (double)y[ks].y
                             : 0.0;
    out[QFT_METRIC_REL_L2] = rn > 0.0 ? dn / rn : dn;
    out[QFT_METRIC_MAX_ERR] = rms > 0.0 ? md / rms : md;
    out[QFT_METRIC_FIDELITY] = (a.cr * a.cr + a.ci * a.ci) / (a.r2 * a.y2);
    out[QFT_METRIC_LEAKAGE] = 1.0 - yk2 / a.y2;
    out[QFT_METRIC_NORM_Y] = yn;
    out[QFT_METRIC_NORM_REF] = rn;
    out[QFT_METRIC_ARGMAX] = a.mri;
  }
}

int compare_parts(int n) {
  const uint64_t N = 1ull << n;
  const uint64_t want = N / 4096;  // about 16 elements per thread
  return (int)(want < 1 ? 1 : (want > 1024 ? 1024 : want));
}

// The separate comparison: one reading pass over y and ref into
// compare_parts(n) partials at `part`, then the finishing workgroup.
hipError_t launch_compare(const void *y, const void *ref, int n, bool c128, double *part,
                          double *metrics, hipStream_t s) {
  const uint64_t N = 1ull << n;
  const int parts = compare_parts(n);
  const uint64_t per = (N + parts - 1) / parts;
  if (c128) {
    hipLaunchKernelGGL(k_compare_part<double>, dim3(parts), dim3(kThreads), 0, s,
                       (const cplx<double> *)y, (const cplx<double> *)ref, N, per, part);
    hipLaunchKernelGGL(k_compare_finish<double>, dim3(1), dim3(kThreads), 0, s,
                       (const cplx<double> *)y, N, part, parts, metrics);
  } else {
    hipLaunchKernelGGL(k_compare_part<float>, dim3(parts), dim3(kThreads), 0, s,
                       (const cplx<float> *)y, (const cplx<float> *)ref, N, per, part);
    hipLaunchKernelGGL(k_compare_finish<float>, dim3(1), dim3(kThreads), 0, s,
                       (const cplx<float> *)y, N, part, parts, metrics);
  }
  return hipGetLastError();
}

// ---- the comparison folded into a plan's last pass ------------------------

// The pass kernels with the comparison epilogue.  A plan's last pass has no
// controls below it, so these have no below-pass diagonal (EXT false).
template <typename Real, int RB>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? (RB >= 5 ? 256 : RB >= 3 ? 512 : 1024)
                                                   : (RB >= 5 ? 512 : 1024))
k_fused_pass_cmp(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  tile_body<Real, RB, true>(d, pass_tile_index(d), in, out,
                            reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x, true);
}

template <typename Real, int NSTL, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_fused_pass2_cmp(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  pass2_tile<Real, 5, NSTL, false, NT, false, true>(
      d, pass_tile_index(d), in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int NSTL, bool NT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_fused_pass2w_cmp(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  pass2_tile<Real, 5, NSTL, false, NT, true, true>(
      d, pass_tile_index(d), in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int S, bool NT>
__global__ void __launch_bounds__(sizeof(Real) == 8 ? 256 : 512)
k_fused_pass3_cmp(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  pass3_tile<Real, 5, S, false, NT, false, true>(
      d, pass_tile_index(d), in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int S, bool NT>
__global__ void QFT_LEAN_BOUNDS(Real)
k_fused_pass3w_cmp(const PassDesc d, const cplx<Real> *in, cplx<Real> *out) {
  extern __shared__ __align__(16) unsigned char qft_smem[];
  pass3_tile<Real, 5, S, false, NT, true, true>(
      d, pass_tile_index(d), in, out, reinterpret_cast<cplx<Real> *>(qft_smem), threadIdx.x);
}

template <typename Real, int RB>
hipError_t launch_cmp_t(const PassLaunch &L, const void *in, void *out, hipStream_t s) {
  using K = void (*)(const PassDesc, const cplx<Real> *, cplx<Real> *);
  K fn = k_fused_pass_cmp<Real, RB>;
  if constexpr (RB == 5) {
    const int shape = pass_kernel_shape(L);
    const bool lean = lean_form(L, sizeof(Real) == 8);
    const int nt = L.d.nt ? 1 : 0;
    if (shape > 16) {
      // the store-exchange shape: the generic kernel (full-tile LDS)
    } else if (shape > 10) {
      static const K tab3[2][3] = {
          {k_fused_pass3_cmp<Real, 1, false>, k_fused_pass3_cmp<Real, 2, false>,
           k_fused_pass3_cmp<Real, 3, false>},
          {k_fused_pass3_cmp<Real, 1, true>, k_fused_pass3_cmp<Real, 2, true>,
           k_fused_pass3_cmp<Real, 3, true>}};
      static const K tab3w[2][3] = {
          {k_fused_pass3w_cmp<Real, 1, false>, k_fused_pass3w_cmp<Real, 2, false>,
           k_fused_pass3w_cmp<Real, 3, false>},
          {k_fused_pass3w_cmp<Real, 1, true>, k_fused_pass3w_cmp<Real, 2, true>,
           k_fused_pass3w_cmp<Real, 3, true>}};
      fn = (lean ? tab3w : tab3)[nt][L.d.lane_swap - 1];
    } else if (shape) {
#define QFT_P2C(K2, N)                                                                \
  {K2<Real, 1, N>, K2<Real, 2, N>, K2<Real, 3, N>, K2<Real, 4, N>, K2<Real, 5, N>}
      static const K tab[2][5] = {QFT_P2C(k_fused_pass2_cmp, false),
                                  QFT_P2C(k_fused_pass2_cmp, true)};
      static const K tabw[2][5] = {QFT_P2C(k_fused_pass2w_cmp, false),
                                   QFT_P2C(k_fused_pass2w_cmp, true)};
#undef QFT_P2C
      fn = (lean ? tabw : tab)[nt][L.d.grp[1].nst - 1];
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

// Partials of the last pass of a fused plan (one per wave, or per thread
// below a wave), and the workgroups that combine them.
uint64_t fused_cmp_parts(const qft_plan_s *p) {
  const PassLaunch &L = p->launches.back();
  return (uint64_t)L.d.ntiles * (uint64_t)norm_parts_per_tile(L.threads);
}
uint32_t fused_cmp_groups(uint64_t parts) {
  const uint64_t g = (parts + kThreads - 1) / kThreads;  // at least a partial per thread
  return (uint32_t)(g < 1 ? 1 : (g > (uint64_t)kMaxCombined ? kMaxCombined : g));
}

size_t execute_compare_ws_bytes(const qft_plan_s *p) {
  if (p->hp.schedule != Schedule::Fused)
    return (size_t)compare_parts(p->hp.n) * kCmpSlots * sizeof(double);
  const uint64_t parts = fused_cmp_parts(p);
  return (size_t)(parts + fused_cmp_groups(parts)) * kCmpSlots * sizeof(double);
}

}  // namespace

namespace qft {

hipError_t launch_fused_pass_compare(const PassLaunch &L, bool c128, const void *in, void *out,
                                     hipStream_t s) {
  if (L.d.ext_tw || !L.d.cmp_ref || !L.d.cmp_part) return hipErrorInvalidValue;
  if (c128) {
    switch (L.d.r) {
      case 1: return launch_cmp_t<double, 1>(L, in, out, s);
      case 2: return launch_cmp_t<double, 2>(L, in, out, s);
      case 3: return launch_cmp_t<double, 3>(L, in, out, s);
      case 4: return launch_cmp_t<double, 4>(L, in, out, s);
      case 5: return launch_cmp_t<double, 5>(L, in, out, s);
    }
  } else {
    switch (L.d.r) {
      case 1: return launch_cmp_t<float, 1>(L, in, out, s);
      case 2: return launch_cmp_t<float, 2>(L, in, out, s);
      case 3: return launch_cmp_t<float, 3>(L, in, out, s);
      case 4: return launch_cmp_t<float, 4>(L, in, out, s);
      case 5: return launch_cmp_t<float, 5>(L, in, out, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace qft

extern "C" {

size_t qft_compare_workspace_bytes(int n) {
  if (n < 0 || n > QFT_MAX_QUBITS) return 0;
  return (size_t)compare_parts(n) * kCmpSlots * sizeof(double);
}

int qft_compare(const void *y, const void *ref, int n, int layout, void *workspace,
                double *metrics_dev, qft_stream_t stream) {
  clear_error();
  if (n < 0 || n > QFT_MAX_QUBITS) return set_error(QFT_ERR_INVALID, "n out of range");
  const bool c128 = (layout & QFT_C128) != 0;
  const size_t es = c128 ? 16 : 8;
  if (!y || !ref || !workspace || !metrics_dev)
    return set_error(QFT_ERR_POINTER, "NULL pointer");
  if ((uintptr_t)y % es || (uintptr_t)ref % es)
    return set_error(QFT_ERR_POINTER, "data pointer is not aligned to the element size");
  if ((uintptr_t)workspace % 8 || (uintptr_t)metrics_dev % 8)
    return set_error(QFT_ERR_POINTER, "workspace or metrics pointer is not 8-byte aligned");
  hipError_t e = launch_compare(y, ref, n, c128, (double *)workspace, metrics_dev,
                                (hipStream_t)stream);
  if (e != hipSuccess)
    return set_error(QFT_ERR_HIP, std::string("compare launch: ") + hipGetErrorString(e));
  return QFT_OK;
}

size_t qft_execute_compare_workspace_bytes(const qft_plan_t *plan) {
  return plan ? execute_compare_ws_bytes(plan) : 0;
}

int qft_execute_compare(qft_plan_t *plan, void *dev_ptr, void *workspace, const void *ref,
                        void *cmp_workspace, double *metrics_dev, qft_stream_t stream) {
  clear_error();
  if (plan && !workspace) workspace = plan->d_ws;
  int rc = check_execute(plan, dev_ptr, workspace);
  if (rc != QFT_OK) return rc;
  const HostPlan &hp = plan->hp;
  if (!ref || !cmp_workspace || !metrics_dev)
    return set_error(QFT_ERR_POINTER, "NULL reference, compare workspace or metrics pointer");
  if ((uintptr_t)ref % hp.elem_bytes)
    return set_error(QFT_ERR_POINTER, "reference pointer is not aligned to the element size");
  if ((uintptr_t)cmp_workspace % 8 || (uintptr_t)metrics_dev % 8)
    return set_error(QFT_ERR_POINTER,
                     "compare workspace or metrics pointer is not 8-byte aligned");
  const uintptr_t bytes = (uintptr_t)hp.elem_bytes << hp.n;
  const uintptr_t r0 = (uintptr_t)ref, d0 = (uintptr_t)dev_ptr;
  if (r0 < d0 + bytes && d0 < r0 + bytes)
    return set_error(QFT_ERR_INVALID, "the reference overlaps the transformed array");
  if (workspace && hp.ws_bytes) {
    // the passes before the last one write the workspace
    const uintptr_t w0 = (uintptr_t)workspace;
    if (r0 < w0 + hp.ws_bytes && w0 < r0 + bytes)
      return set_error(QFT_ERR_INVALID, "the reference overlaps the plan's workspace");
  }
  hipStream_t s = (hipStream_t)stream;
  double *part = (double *)cmp_workspace;
  hipError_t e = hipSuccess;
  if (hp.schedule != Schedule::Fused) {
    rc = enqueue_plan(plan, dev_ptr, workspace, s, nullptr, nullptr, true);
    if (rc != QFT_OK) return rc;
    e = launch_compare(dev_ptr, ref, hp.n, hp.c128, part, metrics_dev, s);
  } else {
    const PassLaunch &last = plan->launches.back();
    if (last.d.ext_tw || last.out_ws)
      return set_error(QFT_ERR_UNSUPPORTED,
                       "the plan's last pass does not end in the data array");
    const FusedCompare cmp{ref, part};
    rc = enqueue_plan(plan, dev_ptr, workspace, s, nullptr, nullptr, true, &cmp);
    if (rc != QFT_OK) return rc;
    const uint64_t parts = fused_cmp_parts(plan);
    const uint32_t groups = fused_cmp_groups(parts);
    const uint64_t per = (parts + groups - 1) / groups;
    double *comb = part + parts * kCmpSlots;
    hipLaunchKernelGGL(k_compare_combine, dim3(groups), dim3(kThreads), 0, s, part, parts, per,
                       comb);
    const uint64_t N = 1ull << hp.n;
    if (hp.c128)
      hipLaunchKernelGGL(k_compare_finish<double>, dim3(1), dim3(kThreads), 0, s,
                         (const cplx<double> *)dev_ptr, N, comb, (int)groups, metrics_dev);
    else
      hipLaunchKernelGGL(k_compare_finish<float>, dim3(1), dim3(kThreads), 0, s,
                         (const cplx<float> *)dev_ptr, N, comb, (int)groups, metrics_dev);
    e = hipGetLastError();
  }
  if (e != hipSuccess)
    return set_error(QFT_ERR_HIP, std::string("compare launch: ") + hipGetErrorString(e));
  return QFT_OK;
}

// 1 - tr with tr = 2^{-M} sum_{y < 2^M} Re prod_{a < M} (1 + e^{i th_a(y)}) / 2,
// th_a(y) = 2 pi (y mod 2^{M-a}) 2^{a-n}: the dropped gates' phase in the
// closed form of the AQFT matrix, summed over the input bits one factor at
// a time.  Each factor is e^{i th/2} cos(th/2), so the term is
// P e^{i Phi} with P = prod cos(th_a/2) and Phi = sum th_a/2, and
// 1 - P cos(Phi) = -expm1(sum log cos(th_a/2)) + 2 P sin^2(Phi/2), which
// keeps its relative accuracy when the error is tiny.
double qft_aqft_expected_error(int n, int cutoff) {
  if (n < 1 || n > 62) return -1.0;
  const int k = (cutoff < 0 || cutoff >= n - 1) ? n - 1 : cutoff;
  const int M = n - 1 - k;
  if (M <= 0) return 0.0;
  if (M > kMaxExpectedBits) return -1.0;
  const uint64_t Y = 1ull << M;
  const double two_pi = 6.283185307179586476925286766559;
  long double acc = 0.0L;
  for (uint64_t y = 0; y < Y; ++y) {
    double logp = 0.0, phi = 0.0;
    for (int a = 0; a < M; ++a) {
      const double th = two_pi * (double)(y & ((1ull << (M - a)) - 1ull)) * ldexp(1.0, a - n);
      const double s = sin(th / 4.0);
      logp += log1p(-2.0 * s * s);  // log cos(th / 2)
      phi += th / 2.0;
    }
    const double P = exp(logp);
    const double sp = sin(phi / 2.0);
    acc += (long double)(-expm1(logp) + 2.0 * P * sp * sp);
  }
  const double one_minus_tr = (double)(acc / (long double)Y);
  return sqrt(2.0 * (one_minus_tr > 0.0 ? one_minus_tr : 0.0));
}

int qft_select_cutoff(int n, double rel_l2_budget) {
  if (n < 1 || n > QFT_MAX_QUBITS || !(rel_l2_budget >= 0.0)) return -1;
  int best = n - 1;
  for (int k = n - 2; k >= 0; --k) {
    const double e = qft_aqft_expected_error(n, k);
    if (e < 0.0 || e > rel_l2_budget) break;
    best = k;
  }
  return best;
}

}  // extern "C"
