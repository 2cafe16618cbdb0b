// Accuracy metrics of a transform against a reference on the device, and the
// closed-form expected error of the range-k AQFT; see include/qft_metrics.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>

#include "../../include/qft_metrics.h"
#include "qft_kernels.h"
#include "qft_runtime.h"

namespace qft {
int set_error(int code, const std::string &msg);
void clear_error();
}  // namespace qft

using namespace qft;

namespace {

constexpr int kThreads = 256;
constexpr int kMaxExpectedBits = 20;  // closed form costs 2^M * M terms
constexpr int kSlots = 8;  // per-workgroup partials, see Part

// interleaved complex element (re, im), as the transforms store it
template <typename Real>
struct alignas(2 * sizeof(Real)) elem {
  Real x, y;
};

// Sums of one workgroup's share (FP64): |y - r|^2, |r|^2, |y|^2,
// Re and Im of conj(r) y, the largest |y - r|^2, and the largest |r|^2 with
// its lowest index.
struct Part {
  double d2, r2, y2, cr, ci, md2, mr2, mri;
};

__device__ __forceinline__ void part_add(Part &a, const Part &b) {
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

__device__ __forceinline__ Part part_shfl_xor(const Part &p, int off) {
  Part q;
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

// Workgroup b reduces the contiguous block [b * per, min(N, (b + 1) * per))
// and writes its Part to part[b].  Each thread sums its elements in index
// order, waves combine lanes in a fixed butterfly, then the 4 wave results
// are combined in order: the result does not depend on scheduling.
template <typename Real>
__global__ void __launch_bounds__(kThreads) k_compare_part(const elem<Real> *y,
                                                           const elem<Real> *r, uint64_t N,
                                                           uint64_t per, double *part) {
  __shared__ Part red[kThreads / 64];
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < N ? lo + per : N;
  Part p{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0.0};
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double yx = (double)y[i].x, yy = (double)y[i].y;
    const double rx = (double)r[i].x, ry = (double)r[i].y;
    const double dx = yx - rx, dy = yy - ry;
    const double d2 = dx * dx + dy * dy;
    const double r2 = rx * rx + ry * ry;
    p.d2 += d2;
    p.r2 += r2;
    p.y2 += yx * yx + yy * yy;
    p.cr += rx * yx + ry * yy;  // conj(r) * y
    p.ci += rx * yy - ry * yx;
    p.md2 = fmax(p.md2, d2);
    if (r2 > p.mr2) {  // indices rise within a thread: first maximum wins
      p.mr2 = r2;
      p.mri = (double)i;
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Part q = part_shfl_xor(p, off);
    // combine in lane order so that every lane holds the same result
    Part lo_p = (threadIdx.x & off) ? q : p;
    const Part hi_p = (threadIdx.x & off) ? p : q;
    part_add(lo_p, hi_p);
    p = lo_p;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = p;
  __syncthreads();
  if (threadIdx.x == 0) {
    Part a = red[0];
    for (int w = 1; w < kThreads / 64; ++w) part_add(a, red[w]);
    double *o = part + (size_t)blockIdx.x * kSlots;
    o[0] = a.d2;
    o[1] = a.r2;
    o[2] = a.y2;
    o[3] = a.cr;
    o[4] = a.ci;
    o[5] = a.md2;
    o[6] = a.mr2;
    o[7] = a.mri;
  }
}

// One workgroup: combine the partials in order, then form the metrics.
template <typename Real>
__global__ void __launch_bounds__(kThreads) k_compare_finish(const elem<Real> *y, uint64_t N,
                                                             const double *part, int nparts,
                                                             double *out) {
  __shared__ Part red[kThreads];
  Part p{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kThreads) {
    const double *o = part + (size_t)b * kSlots;
    const Part q{o[0], o[1], o[2], o[3], o[4], o[5], o[6], o[7]};
    part_add(p, q);
  }
  red[threadIdx.x] = p;
  __syncthreads();
  if (threadIdx.x == 0) {
    Part a = red[0];
    for (int t = 1; t < kThreads; ++t) part_add(a, red[t]);
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

}  // namespace

extern "C" {

size_t qft_compare_workspace_bytes(int n) {
  if (n < 0 || n > QFT_MAX_QUBITS) return 0;
  return (size_t)compare_parts(n) * kSlots * sizeof(double);
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
  const uint64_t N = 1ull << n;
  const int parts = compare_parts(n);
  const uint64_t per = (N + parts - 1) / parts;
  hipStream_t s = (hipStream_t)stream;
  double *part = (double *)workspace;
  if (c128) {
    hipLaunchKernelGGL(k_compare_part<double>, dim3(parts), dim3(kThreads), 0, s,
                       (const elem<double> *)y, (const elem<double> *)ref, N, per, part);
    hipLaunchKernelGGL(k_compare_finish<double>, dim3(1), dim3(kThreads), 0, s,
                       (const elem<double> *)y, N, part, parts, metrics_dev);
  } else {
    hipLaunchKernelGGL(k_compare_part<float>, dim3(parts), dim3(kThreads), 0, s,
                       (const elem<float> *)y, (const elem<float> *)ref, N, per, part);
    hipLaunchKernelGGL(k_compare_finish<float>, dim3(1), dim3(kThreads), 0, s,
                       (const elem<float> *)y, N, part, parts, metrics_dev);
  }
  hipError_t e = hipGetLastError();
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
