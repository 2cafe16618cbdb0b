// Batched uneven-size execution: one persistent launch over (transform,
// pass, tile) work items, captured once per (plans, pointers) set into a HIP
// graph and replayed.  See include/qft.h.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/qft.h"
#include "qft_kernels.h"
#include "qft_runtime.h"

namespace qft {

namespace {

struct BatchEntry {
  std::vector<qft_plan_t *> plans;
  std::vector<void *> ptrs;
  bool c128 = false;
  int maxrb = 1;
  BatchLaunch launch{};
  void *d_mem = nullptr;             // segments, descriptors, io, counters
  std::vector<void *> workspaces;    // one per natural-order multi-pass job
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;

  void release() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    for (void *w : workspaces) hipFree(w);
    if (d_mem) hipFree(d_mem);
    exec = nullptr;
    graph = nullptr;
    d_mem = nullptr;
    workspaces.clear();
  }
};

std::mutex g_mu;
std::vector<BatchEntry *> g_cache;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int build_entry(BatchEntry *e) {
  const int njobs = (int)e->plans.size();
  std::vector<BatchSeg> segs;
  std::vector<PassDesc> descs;
  std::vector<BatchIO> io;
  // per job: resolve its buffers (the state and, for natural-order plans
  // with more than one pass, a workspace owned by this batch entry)
  std::vector<void *> ws(njobs, nullptr);
  int maxP = 0;
  for (int j = 0; j < njobs; ++j) {
    qft_plan_t *p = e->plans[j];
    maxP = std::max(maxP, (int)p->launches.size());
    if (p->hp.ws_bytes) {
      void *w = nullptr;
      hipError_t he = hipMalloc(&w, p->hp.ws_bytes);
      if (he != hipSuccess) return hip_error(he, "batch workspace allocation");
      e->workspaces.push_back(w);
      ws[j] = w;
    }
  }
  uint32_t item = 0;
  int block = 1, lds = 0;
  e->maxrb = 1;
  std::vector<uint32_t> done_before(njobs, 0);
  for (int level = 0; level < maxP; ++level) {
    for (int j = 0; j < njobs; ++j) {
      qft_plan_t *p = e->plans[j];
      if (level >= (int)p->launches.size()) continue;
      const PassLaunch &L = p->launches[level];
      BatchSeg sg;
      sg.first = item;
      sg.ntiles = L.grid;
      sg.desc = (uint32_t)descs.size();
      sg.job = (uint32_t)j;
      sg.wait = done_before[j];
      sg.threads = (uint32_t)L.threads;
      segs.push_back(sg);
      PassDesc d = L.d;
      d.xcd_remap = 0;
      descs.push_back(d);
      BatchIO b;
      b.in = L.in_ws ? ws[j] : e->ptrs[j];
      b.out = L.out_ws ? ws[j] : e->ptrs[j];
      io.push_back(b);
      item += L.grid;
      done_before[j] += L.grid;
      block = std::max(block, L.threads);
      lds = std::max(lds, L.lds_bytes);
      e->maxrb = std::max(e->maxrb, (int)L.d.r);
    }
  }
  if (block > batch_max_block(e->c128, e->maxrb))
    return set_error(QFT_ERR_UNSUPPORTED, "batch mixes tile shapes that do not fit one workgroup size");
  const size_t off_seg = 0;
  const size_t off_desc = align_up(off_seg + segs.size() * sizeof(BatchSeg), 256);
  const size_t off_io = align_up(off_desc + descs.size() * sizeof(PassDesc), 256);
  const size_t off_cnt = align_up(off_io + io.size() * sizeof(BatchIO), 256);
  const size_t bytes = off_cnt + (size_t)(njobs + 2) * sizeof(uint32_t);
  std::vector<unsigned char> host(bytes, 0);
  memcpy(host.data() + off_seg, segs.data(), segs.size() * sizeof(BatchSeg));
  memcpy(host.data() + off_desc, descs.data(), descs.size() * sizeof(PassDesc));
  memcpy(host.data() + off_io, io.data(), io.size() * sizeof(BatchIO));
  hipError_t he = hipMalloc(&e->d_mem, bytes);
  if (he != hipSuccess) return hip_error(he, "batch descriptor allocation");
  he = hipMemcpy(e->d_mem, host.data(), bytes, hipMemcpyHostToDevice);
  if (he != hipSuccess) return hip_error(he, "batch descriptor upload");
  unsigned char *m = (unsigned char *)e->d_mem;
  BatchLaunch &b = e->launch;
  b.segs = (const BatchSeg *)(m + off_seg);
  b.descs = (const PassDesc *)(m + off_desc);
  b.io = (const BatchIO *)(m + off_io);
  b.counters = (uint32_t *)(m + off_cnt);
  b.nseg = (int)segs.size();
  b.njobs = njobs;
  b.total = item;
  b.block = block;
  b.lds_bytes = lds;
  // about 2^26 sleeps of ~128 cycles: far beyond any legal wait, so the
  // limit only ends a wait that could never be met
  b.spin_limit = 1u << 26;
  // persistent grid: the workgroups that fit on the device at once
  int per_cu = 0;
  he = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(e->c128, e->maxrb), block,
                                                    lds);
  if (he != hipSuccess || per_cu < 1) per_cu = 1;
  int cus = 0;
  he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, e->device);
  if (he != hipSuccess || cus < 1) cus = 1;
  b.grid = std::max(1u, std::min<uint32_t>(item, (uint32_t)(per_cu * cus)));
  return QFT_OK;
}

int capture_entry(BatchEntry *e) {
  hipStream_t cs;
  hipError_t he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (he != hipSuccess) return hip_error(he, "capture stream");
  he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    hipError_t le = launch_batch(e->c128, e->maxrb, e->launch, cs);
    he = hipStreamEndCapture(cs, &e->graph);
    if (le != hipSuccess) he = le;
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
  hipStreamDestroy(cs);
  if (he != hipSuccess) return hip_error(he, "batch graph capture");
  return QFT_OK;
}

}  // namespace

void batch_forget_plan(qft_plan_s *plan) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t i = 0; i < g_cache.size();) {
    BatchEntry *e = g_cache[i];
    if (std::find(e->plans.begin(), e->plans.end(), plan) != e->plans.end()) {
      hipDeviceSynchronize();
      e->release();
      delete e;
      g_cache.erase(g_cache.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace qft

using namespace qft;

extern "C" {

int qft_execute_batch_ex(qft_plan_t *const *plans, void *const *dev_ptrs, int count, int flags,
                         qft_stream_t stream) {
  clear_error();
  if (count < 0 || (count > 0 && (!plans || !dev_ptrs)))
    return set_error(QFT_ERR_INVALID, "invalid batch arrays");
  if (count == 0) return QFT_OK;
  if (flags & ~QFT_BATCH_EAGER) return set_error(QFT_ERR_INVALID, "unknown batch flags");
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_error(he, "hipGetDevice");
  bool c128 = false;
  for (int i = 0; i < count; ++i) {
    qft_plan_t *p = plans[i];
    if (!p) return set_error(QFT_ERR_INVALID, "NULL plan in batch");
    if (p->hp.schedule != Schedule::Fused)
      return set_error(QFT_ERR_UNSUPPORTED, "batched execution needs fused-schedule plans");
    if (p->device != dev) return set_error(QFT_ERR_INVALID, "plan belongs to another device");
    if (i == 0) c128 = p->hp.c128;
    if (p->hp.c128 != c128) return set_error(QFT_ERR_UNSUPPORTED, "batch mixes element types");
    if (!dev_ptrs[i]) return set_error(QFT_ERR_POINTER, "NULL data pointer in batch");
    if ((uintptr_t)dev_ptrs[i] % p->hp.elem_bytes)
      return set_error(QFT_ERR_POINTER, "misaligned data pointer in batch");
  }
  std::vector<qft_plan_t *> pv(plans, plans + count);
  std::vector<void *> dv(dev_ptrs, dev_ptrs + count);
  std::lock_guard<std::mutex> lk(g_mu);
  BatchEntry *e = nullptr;
  for (BatchEntry *c : g_cache)
    if (c->device == dev && c->plans == pv && c->ptrs == dv) {
      e = c;
      break;
    }
  if (!e) {
    e = new BatchEntry();
    e->plans = pv;
    e->ptrs = dv;
    e->c128 = c128;
    e->device = dev;
    int rc = build_entry(e);
    if (rc != QFT_OK) {
      e->release();
      delete e;
      return rc;
    }
    g_cache.push_back(e);
  }
  if (flags & QFT_BATCH_EAGER) {
    he = launch_batch(e->c128, e->maxrb, e->launch, (hipStream_t)stream);
    if (he != hipSuccess) return hip_error(he, "batch launch");
    return QFT_OK;
  }
  if (!e->exec) {
    int rc = capture_entry(e);
    if (rc != QFT_OK) return rc;
  }
  he = hipGraphLaunch(e->exec, (hipStream_t)stream);
  if (he != hipSuccess) return hip_error(he, "batch graph launch");
  return QFT_OK;
}

int qft_execute_batch(qft_plan_t *const *plans, void *const *dev_ptrs, int count,
                      qft_stream_t stream) {
  return qft_execute_batch_ex(plans, dev_ptrs, count, 0, stream);
}

int qft_batch_status(qft_plan_t *const *plans, void *const *dev_ptrs, int count) {
  clear_error();
  std::vector<qft_plan_t *> pv(plans, plans + count);
  std::vector<void *> dv(dev_ptrs, dev_ptrs + count);
  std::lock_guard<std::mutex> lk(g_mu);
  for (BatchEntry *c : g_cache) {
    if (c->plans == pv && c->ptrs == dv) {
      uint32_t flag = 0;
      hipError_t he = hipMemcpy(&flag, c->launch.counters + 1 + c->launch.njobs, sizeof(flag),
                                hipMemcpyDeviceToHost);
      if (he != hipSuccess) return hip_error(he, "batch status read");
      if (flag) return set_error(QFT_ERR_HIP, "a batch wait exceeded its spin limit");
      return QFT_OK;
    }
  }
  return set_error(QFT_ERR_INVALID, "no such batch");
}

}  // extern "C"
