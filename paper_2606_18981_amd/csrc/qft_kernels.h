// Launch wrappers for the gfx950 kernels (host-callable, defined in
// qft_kernels.hip).  All return a hipError_t value cast to int.
#pragma once
#include <hip/hip_runtime.h>

#include "qft_internal.h"

namespace qft {

// Let kernel `fn` use up to `bytes` of dynamic LDS (above the 64 KiB
// default) on the current device.  The attribute is per device, so it is set
// once per (device, kernel) pair; thread-safe.
hipError_t ensure_lds_limit(const void *fn, int bytes);

// One fused HBM pass (see qft_internal.h).
hipError_t launch_fused_pass(const PassLaunch &L, bool c128, const void *in, void *out,
                             hipStream_t s);

// The last pass of a plan with its output also compared with L.d.cmp_ref
// (the pass kernels' comparison epilogue; defined in qft_metrics.hip).  The
// last pass has no controls below it: L.d.ext_tw must be 0.
hipError_t launch_fused_pass_compare(const PassLaunch &L, bool c128, const void *in, void *out,
                                     hipStream_t s);

// Batched launches (see k_batch_group).
struct BatchSeg {
  uint32_t first;    // first work item (workgroup) of the segment in its group
  uint32_t ntiles;   // tiles (items) in the segment
  uint32_t desc;     // index into the descriptor / io arrays
  uint32_t job;      // transform index
};
struct BatchIO {
  const void *in;
  void *out;
};
// one launch: the segments [segs, segs + nseg) of a (pass level, radix,
// workgroup size) group
struct BatchGroup {
  const BatchSeg *segs;
  const PassDesc *descs;
  const BatchIO *io;
  int nseg;
  uint32_t items;
  int threads;
  int lds_bytes;
  int r;
  int shape;  // fused_pass_shape of every pass in the group
};
hipError_t launch_batch_group(bool c128, const BatchGroup &g, hipStream_t s);

// Kernel of a pass (pass_kernel_shape): 0 for the generic pass kernel;
// 1..10 for the compile-time two-group kernel (radix 32, the first group
// full, the last holding pass bit 0); 11..16 for the compile-time
// three-group kernel (the last group reached by cross-lane swaps); 17..21
// for the two-group kernel that stores through an exchange-only third group.
int fused_pass_shape(const PassLaunch &L);

// Gate-by-gate sweeps (unfused circuit, Fig. 1).
hipError_t launch_h(void *psi, int n, int t, bool c128, hipStream_t s);
hipError_t launch_cphase(void *psi, int n, int c, int t, double re, double im, bool c128,
                         hipStream_t s);
hipError_t launch_swap(void *psi, int n, int a, int b, bool c128, hipStream_t s);
hipError_t launch_scale(void *psi, int n, double f, bool c128, hipStream_t s);

// Input norm: partial sums of |x|^2 over `nparts` contiguous blocks, and
// out[0] = sqrt(sum of `count` partials) in FP64.
hipError_t launch_norm_sweep(const void *psi, int n, bool c128, double *part, uint32_t nparts,
                             hipStream_t s);
hipError_t launch_norm_finish(const double *part, uint32_t count, double *out, hipStream_t s);

// Philox-4x32-10 input generator.
// dst[i] = i < count ? src[i] : 0 for i < 2^n.
hipError_t launch_pad(const void *src, size_t count, void *dst, int n, bool c128, hipStream_t s);

hipError_t launch_fill_random(void *psi, int n, bool c128, int dist, uint64_t seed,
                              uint64_t stream_id, hipStream_t s);

}  // namespace qft
