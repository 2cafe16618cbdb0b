// Launch wrappers for the gfx950 kernels (host-callable, defined in
// qft_kernels.hip).  All return a hipError_t value cast to int.
#pragma once
#include <hip/hip_runtime.h>

#include "qft_internal.h"

namespace qft {

// One fused HBM pass (see qft_internal.h).
hipError_t launch_fused_pass(const PassLaunch &L, bool c128, const void *in, void *out,
                             hipStream_t s);

// Persistent batch launch (see k_batch).
struct BatchSeg {
  uint32_t first;    // first work item of the segment
  uint32_t ntiles;   // tiles (items) in the segment
  uint32_t desc;     // index into the descriptor / io arrays
  uint32_t job;      // transform index
  uint32_t wait;     // finished tiles of the job required before starting
  uint32_t threads;  // active threads per tile
};
struct BatchIO {
  const void *in;
  void *out;
};
struct BatchLaunch {
  const BatchSeg *segs;
  const PassDesc *descs;
  const BatchIO *io;
  uint32_t *counters;  // njobs + 2 words
  int nseg;
  int njobs;
  uint32_t total;
  uint32_t grid;
  int block;
  int lds_bytes;
  uint32_t spin_limit;
};
hipError_t launch_batch(bool c128, int maxrb, const BatchLaunch &b, hipStream_t s);
const void *batch_kernel(bool c128, int maxrb);
int batch_max_block(bool c128, int maxrb);

// Gate-by-gate sweeps (unfused circuit, Fig. 1).
hipError_t launch_h(void *psi, int n, int t, bool c128, hipStream_t s);
hipError_t launch_cphase(void *psi, int n, int c, int t, double re, double im, bool c128,
                         hipStream_t s);
hipError_t launch_swap(void *psi, int n, int a, int b, bool c128, hipStream_t s);
hipError_t launch_scale(void *psi, int n, double f, bool c128, hipStream_t s);

// Philox-4x32-10 input generator.
hipError_t launch_fill_random(void *psi, int n, bool c128, int dist, uint64_t seed,
                              uint64_t stream_id, hipStream_t s);

}  // namespace qft
