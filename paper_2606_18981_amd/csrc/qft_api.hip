// C ABI of libqft.so: plan / execute / destroy, plan description, per-pass
// timing and the device input generator.  See include/qft.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qft.h"
#include "qft_kernels.h"
#include "qft_planner.h"
#include "qft_runtime.h"

// Partial sums of |x|^2 for qft_execute_norm_static: file-scope device
// memory instead of a plan-owned hipMalloc'd buffer, so that entry point
// allocates nothing.  Each GPU the library runs on holds its own copy
// (QFT_NORM_SCRATCH_DOUBLES doubles, 8 MiB) until the process ends.  In host
// code the name `scratch` is only a host-side stand-in: the device address
// comes from hipGetSymbolAddress, once per device, and only that address is
// passed to kernels.
static __device__ __align__(256) double scratch[QFT_NORM_SCRATCH_DOUBLES];

namespace {
thread_local std::string g_last_error;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this device's scratch array (resolved on the first call
// on the device, with the device current).
int scratch_address(int dev, double **out) {
  if (dev < 0 || dev >= kMaxScratchDevices)
    return qft::set_error(QFT_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return qft::hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                            "hipGetSymbolAddress(scratch)");
    }
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return QFT_OK;
}
}

namespace qft {

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_error(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? QFT_ERR_NOMEM : QFT_ERR_HIP;
}

void clear_error() { g_last_error.clear(); }

// Enqueue the kernels of a plan.  `ws` may be NULL when the plan needs none.
// With norm_out, `part` holds the plan's norm_parts_for() partial sums.
// With cmp (fused schedule only), the last pass also writes the comparison
// partials of its output against cmp->ref.
int enqueue_plan(qft_plan_s *p, void *dev, void *ws, hipStream_t s, double *norm_out,
                 double *part, bool allow_timing, const FusedCompare *cmp) {
  const HostPlan &hp = p->hp;
  hipError_t e = hipSuccess;
  size_t li = 0;
  const bool timing = p->timing && allow_timing;
  auto mark = [&](size_t i) -> hipError_t {
    return timing ? hipEventRecord(p->timer.slot(i), s) : hipSuccess;
  };
  const uint32_t nparts = norm_out ? norm_parts_for(p) : 0;
  if (norm_out && hp.schedule == Schedule::Gates) {
    e = launch_norm_sweep(dev, hp.n, hp.c128, part, nparts, s);
    if (e != hipSuccess) return hip_error(e, "norm sweep launch");
  }
  if (timing && (e = p->timer.begin(p->num_launches())) != hipSuccess)
    return hip_error(e, "timing events");
  if (hp.schedule == Schedule::Fused) {
    for (size_t i = 0; i < p->launches.size(); ++i) {
      const PassLaunch &L = p->launches[i];
      if ((e = mark(li)) != hipSuccess) return hip_error(e, "timing event record");
      const void *in = L.in_ws ? ws : dev;
      void *out = L.out_ws ? ws : dev;
      const bool first_norm = i == 0 && norm_out;
      const bool last_cmp = i + 1 == p->launches.size() && cmp;
      if (first_norm || last_cmp) {
        // the first pass also sums |x|^2 of the tiles it loads; the last
        // also compares the tiles it stores with the reference
        PassLaunch Lx = L;
        if (first_norm) Lx.d.norm_part = part;
        if (last_cmp) {
          Lx.d.cmp_ref = cmp->ref;
          Lx.d.cmp_part = cmp->part;
          e = launch_fused_pass_compare(Lx, hp.c128, in, out, s);
        } else {
          e = launch_fused_pass(Lx, hp.c128, in, out, s);
        }
      } else {
        e = launch_fused_pass(L, hp.c128, in, out, s);
      }
      if (e != hipSuccess) return hip_error(e, "fused pass launch");
      ++li;
    }
  } else {
    for (const Gate &g : hp.gates) {
      if ((e = mark(li)) != hipSuccess) return hip_error(e, "timing event record");
      if (g.kind == 0) e = launch_h(dev, hp.n, g.a, hp.c128, s);
      else if (g.kind == 1) e = launch_cphase(dev, hp.n, g.a, g.b, g.re, g.im, hp.c128, s);
      else e = launch_swap(dev, hp.n, g.a, g.b, hp.c128, s);
      if (e != hipSuccess) return hip_error(e, "gate sweep launch");
      ++li;
    }
    if (hp.gate_norm != 1.0) {
      if ((e = mark(li)) != hipSuccess) return hip_error(e, "timing event record");
      e = launch_scale(dev, hp.n, hp.gate_norm, hp.c128, s);
      if (e != hipSuccess) return hip_error(e, "scale launch");
      ++li;
    }
  }
  if ((e = mark(li)) != hipSuccess) return hip_error(e, "timing event record");
  if (timing) p->timer.end();
  if (norm_out) {
    e = launch_norm_finish(part, nparts, norm_out, s);
    if (e != hipSuccess) return hip_error(e, "norm launch");
  }
  return QFT_OK;
}

uint32_t norm_parts_for(const qft_plan_s *p) {
  const HostPlan &hp = p->hp;
  if (hp.schedule == Schedule::Fused) {
    const PassLaunch &L = p->launches[0];
    return L.d.ntiles * (uint32_t)norm_parts_per_tile(L.threads);
  }
  const uint32_t N = 1u << hp.n;
  return std::max(1u, std::min(1024u, N / 4096u));
}

// Argument checks shared by the execute entry points (no device work).
int check_execute(qft_plan_s *plan, void *dev_ptr, void *workspace) {
  if (!plan) return set_error(QFT_ERR_INVALID, "plan is NULL");
  if (!dev_ptr) return set_error(QFT_ERR_POINTER, "data pointer is NULL");
  if ((uintptr_t)dev_ptr % plan->hp.elem_bytes)
    return set_error(QFT_ERR_POINTER, "data pointer is not aligned to the element size");
  if (plan->hp.ws_bytes && !workspace)
    return set_error(QFT_ERR_POINTER,
                     "this plan needs a workspace (pass one with qft_execute_ws)");
  if (workspace && (uintptr_t)workspace % plan->hp.elem_bytes)
    return set_error(QFT_ERR_POINTER, "workspace pointer is not aligned to the element size");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  if (dev != plan->device)
    return set_error(QFT_ERR_INVALID, "the current device is not the plan's device");
  return QFT_OK;
}

// ---- per-launch timing ---------------------------------------------------

hipEvent_t LaunchTimer::slot(size_t i) { return events[cur_base + i]; }

hipError_t LaunchTimer::begin(int launches) {
  nl = launches;
  const size_t need = (size_t)(execs + 1) * (size_t)(launches + 1);
  while (events.size() < need) {
    hipEvent_t ev;
    const hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    events.push_back(ev);
  }
  cur_base = (size_t)execs * (size_t)(launches + 1);
  return hipSuccess;
}

void LaunchTimer::end() { ++execs; }

void LaunchTimer::release() {
  for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
  events.clear();
  execs = 0;
}

}  // namespace qft

using namespace qft;

static qft_plan_t *make_plan(int n, int cutoff, int norm, int layout, const qft_config_t *cfg) {
  clear_error();
  qft_plan_t *p = new (std::nothrow) qft_plan_s();
  if (!p) {
    set_error(QFT_ERR_NOMEM, "host allocation failed");
    return nullptr;
  }
  std::string err;
  qft_config_t tuned;
  // the tuning table only when asked for (QFT_PLAN_TUNED), so that a plan
  // does not depend on what the process tuned before
  if (!cfg && (layout & QFT_PLAN_TUNED) && !(layout & QFT_SCHEDULE_GATES) &&
      tune_table_lookup(n, cutoff, layout, &tuned))
    cfg = &tuned;
  int rc = build_host_plan(n, cutoff, norm, layout, cfg, p->hp, err);
  if (rc != QFT_OK) {
    set_error(rc, err);
    delete p;
    return nullptr;
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    hip_error(e, "hipGetDevice");
    delete p;
    return nullptr;
  }
  HostPlan &hp = p->hp;
  if (!hp.tables.empty()) {
    e = hipMalloc(&p->d_tables, hp.tables.size());
    if (e != hipSuccess) {
      hip_error(e, "table allocation");
      delete p;
      return nullptr;
    }
    e = hipMemcpy(p->d_tables, hp.tables.data(), hp.tables.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      hip_error(e, "table upload");
      (void)hipFree(p->d_tables);
      delete p;
      return nullptr;
    }
  }
  if (hp.ws_bytes && !(layout & QFT_PLAN_NO_WORKSPACE)) {
    e = hipMalloc(&p->d_ws, hp.ws_bytes);
    if (e != hipSuccess) {
      hip_error(e, "workspace allocation");
      if (p->d_tables) (void)hipFree(p->d_tables);
      delete p;
      return nullptr;
    }
  }
  p->launches = hp.passes;
  for (size_t i = 0; i < p->launches.size(); ++i) {
    PassLaunch &L = p->launches[i];
    unsigned char *t = (unsigned char *)p->d_tables;
    L.d.tw_int = t + hp.off_int;
    L.d.tw_lo = t + hp.off_lo;
    L.d.tw_hi = t + hp.off_hi;
    L.d.gtab = hp.off_gtab[i] ? t + hp.off_gtab[i] : nullptr;
    L.d.gtab1 = hp.off_gtab1[i] ? t + hp.off_gtab1[i] : nullptr;
  }
  return p;
}

extern "C" {

qft_plan_t *qft_plan(int n, int cutoff, int norm, int layout) {
  return make_plan(n, cutoff, norm, layout, nullptr);
}

qft_plan_t *qft_plan_config(int n, int cutoff, int norm, int layout, const qft_config_t *config) {
  return make_plan(n, cutoff, norm, layout, config);
}

int qft_execute_ws(qft_plan_t *plan, void *dev_ptr, void *workspace, qft_stream_t stream) {
  clear_error();
  int rc = check_execute(plan, dev_ptr, workspace);
  if (rc != QFT_OK) return rc;
  return enqueue_plan(plan, dev_ptr, workspace, (hipStream_t)stream, nullptr, nullptr, true);
}

int qft_execute_norm(qft_plan_t *plan, void *dev_ptr, void *workspace, double *norm_dev,
                     qft_stream_t stream) {
  clear_error();
  if (plan && !workspace) workspace = plan->d_ws;
  int rc = check_execute(plan, dev_ptr, workspace);
  if (rc != QFT_OK) return rc;
  if (!norm_dev) return set_error(QFT_ERR_POINTER, "norm pointer is NULL");
  if ((uintptr_t)norm_dev % sizeof(double))
    return set_error(QFT_ERR_POINTER, "norm pointer is not aligned to 8 bytes");
  if (!plan->d_norm) {
    const uint32_t parts = norm_parts_for(plan);
    hipError_t e = hipMalloc(&plan->d_norm, (size_t)parts * sizeof(double));
    if (e != hipSuccess) {
      plan->d_norm = nullptr;
      (void)hipGetLastError();
      return set_error(QFT_ERR_NOMEM, "cannot allocate the norm partial sums");
    }
    plan->norm_parts = parts;
  }
  return enqueue_plan(plan, dev_ptr, workspace, (hipStream_t)stream, norm_dev, plan->d_norm,
                      true);
}

int qft_execute_norm_static(qft_plan_t *plan, void *dev_ptr, void *workspace, double *norm_dev,
                            qft_stream_t stream) {
  clear_error();
  if (plan && !workspace) workspace = plan->d_ws;
  int rc = check_execute(plan, dev_ptr, workspace);
  if (rc != QFT_OK) return rc;
  if (!norm_dev) return set_error(QFT_ERR_POINTER, "norm pointer is NULL");
  if ((uintptr_t)norm_dev % sizeof(double))
    return set_error(QFT_ERR_POINTER, "norm pointer is not aligned to 8 bytes");
  const uint32_t parts = norm_parts_for(plan);
  if (parts > QFT_NORM_SCRATCH_DOUBLES)
    return set_error(QFT_ERR_UNSUPPORTED,
                     "this plan needs more norm partial sums than the static scratch holds "
                     "(QFT_NORM_SCRATCH_DOUBLES); use qft_execute_norm");
  double *part = nullptr;
  rc = scratch_address(plan->device, &part);
  if (rc != QFT_OK) return rc;
  // every partial is written by the first pass (or the norm sweep) before the
  // final sum reads it, so the scratch needs no clearing between calls
  return enqueue_plan(plan, dev_ptr, workspace, (hipStream_t)stream, norm_dev, part, false);
}

int qft_execute(qft_plan_t *plan, void *dev_ptr, qft_stream_t stream) {
  if (!plan) {
    clear_error();
    return set_error(QFT_ERR_INVALID, "plan is NULL");
  }
  return qft_execute_ws(plan, dev_ptr, plan->d_ws, stream);
}

void qft_destroy(qft_plan_t *plan) {
  if (!plan) return;
  batch_forget_plan(plan);
  plan->timer.release();
  if (plan->d_tables) (void)hipFree(plan->d_tables);
  if (plan->d_ws) (void)hipFree(plan->d_ws);
  if (plan->d_norm) (void)hipFree(plan->d_norm);
  delete plan;
}

const char *qft_last_error(void) { return g_last_error.c_str(); }

int qft_plan_info(const qft_plan_t *plan, qft_plan_info_t *out) {
  clear_error();
  if (!plan || !out) return set_error(QFT_ERR_INVALID, "NULL argument");
  describe_plan(plan->hp, out);
  return QFT_OK;
}

size_t qft_plan_device_bytes(const qft_plan_t *plan) {
  if (!plan) return 0;
  const HostPlan &hp = plan->hp;
  return hp.tables.size() + (plan->d_ws ? hp.ws_bytes : 0) +
         (plan->d_norm ? (size_t)plan->norm_parts * sizeof(double) : 0);
}

int qft_plan_describe(int n, int cutoff, int norm, int layout, const qft_config_t *config,
                      qft_plan_info_t *out) {
  clear_error();
  if (!out) return set_error(QFT_ERR_INVALID, "NULL argument");
  HostPlan hp;
  std::string err;
  int rc = build_host_plan(n, cutoff, norm, layout, config, hp, err);
  if (rc != QFT_OK) return set_error(rc, err);
  describe_plan(hp, out);
  return QFT_OK;
}

int qft_plan_set_timing(qft_plan_t *plan, int enable) {
  clear_error();
  if (!plan) return set_error(QFT_ERR_INVALID, "plan is NULL");
  plan->timing = enable != 0;
  return QFT_OK;
}

int qft_plan_pass_times(qft_plan_t *plan, double *ms, int max, long long *execs) {
  clear_error();
  if (!plan) return set_error(QFT_ERR_INVALID, "plan is NULL");
  LaunchTimer &t = plan->timer;
  const int nl = plan->num_launches();
  std::vector<double> acc(nl, 0.0);
  if (t.execs > 0) {
    hipError_t e = hipEventSynchronize(t.events[(size_t)t.execs * (nl + 1) - 1]);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
    for (long long x = 0; x < t.execs; ++x) {
      for (int i = 0; i < nl; ++i) {
        float f = 0.f;
        e = hipEventElapsedTime(&f, t.events[(size_t)x * (nl + 1) + i],
                                t.events[(size_t)x * (nl + 1) + i + 1]);
        if (e != hipSuccess) return hip_error(e, "hipEventElapsedTime");
        acc[i] += f;
      }
    }
  }
  if (ms)
    for (int i = 0; i < nl && i < max; ++i) ms[i] = t.execs ? acc[i] / (double)t.execs : 0.0;
  if (execs) *execs = t.execs;
  t.execs = 0;
  return QFT_OK;
}

int qft_qubits_for(size_t count) {
  if (count == 0) return -1;
  int n = 0;
  while (n < 63 && ((size_t)1 << n) < count) ++n;
  return n <= QFT_MAX_QUBITS ? n : -1;
}

int qft_pad(const void *src, size_t count, void *dst, int n, int layout, qft_stream_t stream) {
  clear_error();
  if (n < 0 || n > QFT_MAX_QUBITS) return set_error(QFT_ERR_INVALID, "n out of range");
  if (count > ((size_t)1 << n)) return set_error(QFT_ERR_INVALID, "count exceeds 2^n");
  const bool c128 = (layout & QFT_C128) != 0;
  const size_t es = c128 ? 16 : 8;
  if (!dst || (count && !src)) return set_error(QFT_ERR_POINTER, "NULL pointer");
  if ((uintptr_t)dst % es || (uintptr_t)src % es)
    return set_error(QFT_ERR_POINTER, "pointer is not aligned to the element size");
  const uintptr_t s0 = (uintptr_t)src, s1 = s0 + count * es;
  const uintptr_t d0 = (uintptr_t)dst, d1 = d0 + (es << n);
  if (count && s0 < d1 && d0 < s1) return set_error(QFT_ERR_INVALID, "src and dst overlap");
  hipError_t e = launch_pad(src, count, dst, n, c128, (hipStream_t)stream);
  if (e != hipSuccess) return hip_error(e, "pad launch");
  return QFT_OK;
}

int qft_fill_random(void *dev_ptr, int n, int layout, int dist, uint64_t seed, uint64_t stream_id,
                    qft_stream_t stream) {
  clear_error();
  if (n < 1 || n > QFT_MAX_QUBITS) return set_error(QFT_ERR_INVALID, "n out of range");
  if (dist != QFT_RNG_GAUSSIAN && dist != QFT_RNG_UNIFORM)
    return set_error(QFT_ERR_INVALID, "unknown distribution");
  if (!dev_ptr) return set_error(QFT_ERR_POINTER, "data pointer is NULL");
  const bool c128 = (layout & QFT_C128) != 0;
  if ((uintptr_t)dev_ptr % (c128 ? 16 : 8))
    return set_error(QFT_ERR_POINTER, "data pointer is not aligned to the element size");
  hipError_t e = launch_fill_random(dev_ptr, n, c128, dist, seed, stream_id, (hipStream_t)stream);
  if (e != hipSuccess) return hip_error(e, "fill_random launch");
  return QFT_OK;
}

}  // extern "C"
