// Batched uneven-size execution: the tiles of all transforms, launched pass
// level by pass level (one launch per level, radix, workgroup size and
// kernel shape), captured once per (plans, pointers) set into a HIP graph
// and replayed.  Transforms of one pass depend on nothing: their launches go
// to a stream of their own, forked at the start and joined at the end, and
// run beside the others.  The passes of multi-pass transforms are aligned to
// the last levels (a transform of P passes runs its pass p at level
// maxP - P + p).  See include/qft.h.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <mutex>
#include <vector>

#include "../../include/qft.h"
#include "qft_kernels.h"
#include "qft_runtime.h"

namespace qft {

namespace {

// The groups of one pass level touch different transforms, so they may run
// at the same time: on up to kLevelStreams streams (the caller's and side
// streams of the batch entry), joined again before the next level; one more
// side stream runs the one-pass transforms.  (Four streams: the hardware
// queues a process gets by default.)
constexpr int kForkStreams = 4;
constexpr int kLevelStreams = kForkStreams - 1;
// launch cost model for dealing a level's groups to streams: bytes moved at
// this rate, but at least this latency per launch
constexpr double kGroupBytesPerUs = 4.0e6;
constexpr double kLaunchFloorUs = 10.0;

// Cached (plans, pointers) sets, each with its graph, workspaces, streams
// and events; beyond this many the oldest is released.
constexpr size_t kMaxCachedSets = 64;

struct BatchEntry {
  std::vector<qft_plan_t *> plans;
  std::vector<void *> ptrs;
  bool c128 = false;
  std::vector<BatchGroup> groups;    // launch order: pass level by pass level
  void *d_mem = nullptr;             // segments, descriptors, io
  std::vector<void *> workspaces;    // one per natural-order multi-pass job
  std::vector<int> levels;           // pass level of each group; -1: one-pass
  std::vector<double> cost;          // modelled time of each group (us)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
  // side streams (default priority) and events for the fork / join of the
  // groups of one level
  hipStream_t side[kForkStreams - 1] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kForkStreams - 1] = {};

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void *w : workspaces) (void)hipFree(w);
    if (d_mem) (void)hipFree(d_mem);
    for (hipStream_t &st : side) {
      if (st) (void)hipStreamDestroy(st);
      st = nullptr;
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    fork_ev = nullptr;
    for (hipEvent_t &ev : join_ev) {
      if (ev) (void)hipEventDestroy(ev);
      ev = nullptr;
    }
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
  std::vector<PassDesc> descs;
  std::vector<BatchIO> io;
  // per job: its buffers (the state and, for natural-order plans with more
  // than one pass, a workspace owned by this batch entry)
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
  // group the (job, pass) launches by pass level, radix and workgroup size
  struct GroupBuild {
    int level, r, threads, lds, shape;
    std::vector<BatchSeg> segs;
    uint32_t items = 0;
  };
  std::vector<GroupBuild> gb;
  // level -1: the one-pass transforms; then the pass levels of the others
  for (int level = -1; level < maxP; ++level) {
    std::map<std::tuple<int, int, int>, size_t> index;  // (r, threads, shape) -> group
    for (int j = 0; j < njobs; ++j) {
      qft_plan_t *p = e->plans[j];
      const int P = (int)p->launches.size();
      int pass;
      if (level < 0) pass = P == 1 ? 0 : -1;
      else pass = P == 1 ? -1 : level - (maxP - P);  // right-aligned: the last pass at the last level
      if (pass < 0) continue;
      const PassLaunch &L = p->launches[pass];
      const int shape = fused_pass_shape(L);
      const auto key = std::make_tuple((int)L.d.r, L.threads, shape);
      auto it = index.find(key);
      if (it == index.end()) {
        GroupBuild g;
        g.level = level;
        g.r = L.d.r;
        g.threads = L.threads;
        g.shape = shape;
        g.lds = 0;
        gb.push_back(g);
        it = index.emplace(key, gb.size() - 1).first;
      }
      GroupBuild &g = gb[it->second];
      BatchSeg sg;
      sg.first = g.items;
      sg.ntiles = L.d.ntiles;
      sg.desc = (uint32_t)descs.size();
      sg.job = (uint32_t)j;
      g.segs.push_back(sg);
      g.items += L.d.ntiles;
      g.lds = std::max(g.lds, L.lds_bytes);
      PassDesc d = L.d;
      d.xcd_remap = 0;
      descs.push_back(d);
      BatchIO b;
      b.in = L.in_ws ? ws[j] : e->ptrs[j];
      b.out = L.out_ws ? ws[j] : e->ptrs[j];
      io.push_back(b);
    }
  }
  size_t nsegs = 0;
  for (const GroupBuild &g : gb) nsegs += g.segs.size();
  const size_t off_seg = 0;
  const size_t off_desc = align_up(off_seg + nsegs * sizeof(BatchSeg), 256);
  const size_t off_io = align_up(off_desc + descs.size() * sizeof(PassDesc), 256);
  const size_t bytes = off_io + io.size() * sizeof(BatchIO);
  std::vector<unsigned char> host(bytes, 0);
  size_t seg_at = 0;
  std::vector<size_t> seg_start;
  for (const GroupBuild &g : gb) {
    seg_start.push_back(seg_at);
    memcpy(host.data() + off_seg + seg_at * sizeof(BatchSeg), g.segs.data(),
           g.segs.size() * sizeof(BatchSeg));
    seg_at += g.segs.size();
  }
  memcpy(host.data() + off_desc, descs.data(), descs.size() * sizeof(PassDesc));
  memcpy(host.data() + off_io, io.data(), io.size() * sizeof(BatchIO));
  hipError_t he = hipMalloc(&e->d_mem, bytes);
  if (he != hipSuccess) return hip_error(he, "batch descriptor allocation");
  he = hipMemcpy(e->d_mem, host.data(), bytes, hipMemcpyHostToDevice);
  if (he != hipSuccess) return hip_error(he, "batch descriptor upload");
  unsigned char *m = (unsigned char *)e->d_mem;
  for (size_t i = 0; i < gb.size(); ++i) {
    BatchGroup g;
    g.segs = (const BatchSeg *)(m + off_seg) + seg_start[i];
    g.descs = (const PassDesc *)(m + off_desc);
    g.io = (const BatchIO *)(m + off_io);
    g.nseg = (int)gb[i].segs.size();
    g.items = gb[i].items;
    g.threads = gb[i].threads;
    g.lds_bytes = gb[i].lds;
    g.r = gb[i].r;
    g.shape = gb[i].shape;
    e->groups.push_back(g);
    e->levels.push_back(gb[i].level);
    const double bytes = 2.0 * (double)g.items * (double)g.threads * (double)(1 << g.r) *
                         (e->c128 ? 16.0 : 8.0);
    e->cost.push_back(std::max(kLaunchFloorUs, bytes / kGroupBytesPerUs));
  }
  for (hipStream_t &st : e->side) {
    he = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (he != hipSuccess) {
      st = nullptr;
      return hip_error(he, "batch side stream");
    }
  }
  he = hipEventCreateWithFlags(&e->fork_ev, hipEventDisableTiming);
  if (he != hipSuccess) {
    e->fork_ev = nullptr;
    return hip_error(he, "batch event");
  }
  for (hipEvent_t &ev : e->join_ev) {
    he = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (he != hipSuccess) {
      ev = nullptr;
      return hip_error(he, "batch event");
    }
  }
  return QFT_OK;
}

// Level by level: a level with one group runs on `s`; the groups of a wider
// level are dealt, largest modelled cost first, each to the stream of the
// level with the least cost so far (`s` and the first side streams), which
// wait for `s` before and are waited for by `s` after.  The one-pass groups
// (level -1) run on the last side stream, forked from `s` at the start and
// joined at the end; they are enqueued after the first level's launches (a
// graph dispatches its kernels in the order they were captured, and the
// large first passes should start first).  Under graph capture the same
// calls record the forks and joins as graph edges.
hipError_t launch_entry(BatchEntry *e, hipStream_t s) {
  const size_t ng = e->groups.size();
  hipError_t he;
  hipStream_t free_st = e->side[kForkStreams - 2];
  size_t nfree = 0;
  while (nfree < ng && e->levels[nfree] < 0) ++nfree;
  bool free_done = nfree == 0;
  if (!free_done) {
    he = hipEventRecord(e->fork_ev, s);
    if (he != hipSuccess) return he;
    he = hipStreamWaitEvent(free_st, e->fork_ev, 0);
    if (he != hipSuccess) return he;
  }
  auto launch_free = [&]() -> hipError_t {
    for (size_t k = 0; k < nfree; ++k) {
      hipError_t h = launch_batch_group(e->c128, e->groups[k], free_st);
      if (h != hipSuccess) return h;
    }
    free_done = true;
    return hipSuccess;
  };
  size_t i = nfree;
  while (i < ng) {
    size_t j = i;
    while (j < ng && e->levels[j] == e->levels[i]) ++j;
    if (j - i == 1) {
      he = launch_batch_group(e->c128, e->groups[i], s);
      if (he != hipSuccess) return he;
      if (!free_done && (he = launch_free()) != hipSuccess) return he;
      i = j;
      continue;
    }
    std::vector<size_t> order;
    for (size_t k = i; k < j; ++k) order.push_back(k);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return e->cost[a] > e->cost[b]; });
    const int used = (int)std::min<size_t>(order.size(), kLevelStreams);
    he = hipEventRecord(e->fork_ev, s);
    if (he != hipSuccess) return he;
    for (int k = 1; k < used; ++k) {
      he = hipStreamWaitEvent(e->side[k - 1], e->fork_ev, 0);
      if (he != hipSuccess) return he;
    }
    double load[kLevelStreams] = {};
    for (size_t k = 0; k < order.size(); ++k) {
      int lane = 0;
      for (int q = 1; q < used; ++q)
        if (load[q] < load[lane]) lane = q;
      load[lane] += e->cost[order[k]];
      hipStream_t st = lane == 0 ? s : e->side[lane - 1];
      he = launch_batch_group(e->c128, e->groups[order[k]], st);
      if (he != hipSuccess) return he;
    }
    if (!free_done && (he = launch_free()) != hipSuccess) return he;
    for (int k = 1; k < used; ++k) {
      he = hipEventRecord(e->join_ev[k - 1], e->side[k - 1]);
      if (he != hipSuccess) return he;
      he = hipStreamWaitEvent(s, e->join_ev[k - 1], 0);
      if (he != hipSuccess) return he;
    }
    i = j;
  }
  if (nfree > 0) {
    if (!free_done && (he = launch_free()) != hipSuccess) return he;
    he = hipEventRecord(e->join_ev[kForkStreams - 2], free_st);
    if (he != hipSuccess) return he;
    he = hipStreamWaitEvent(s, e->join_ev[kForkStreams - 2], 0);
    if (he != hipSuccess) return he;
  }
  return hipSuccess;
}

int capture_entry(BatchEntry *e) {
  hipStream_t cs;
  hipError_t he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (he != hipSuccess) return hip_error(he, "capture stream");
  he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    hipError_t le = launch_entry(e, cs);
    he = hipStreamEndCapture(cs, &e->graph);
    if (le != hipSuccess) he = le;
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (he != hipSuccess) return hip_error(he, "batch graph capture");
  return QFT_OK;
}

}  // namespace

void batch_forget_plan(qft_plan_s *plan) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t i = 0; i < g_cache.size();) {
    BatchEntry *e = g_cache[i];
    if (std::find(e->plans.begin(), e->plans.end(), plan) != e->plans.end()) {
      // (a device error here is sticky: the caller's next call reports it)
      (void)hipDeviceSynchronize();
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
    if (g_cache.size() >= kMaxCachedSets) {
      // the oldest set may still run on some stream: wait for the device
      // before its graph, workspaces and streams are released
      const hipError_t he = hipDeviceSynchronize();
      if (he != hipSuccess) {
        e->release();
        delete e;
        return hip_error(he, "batch cache eviction");
      }
      g_cache.front()->release();
      delete g_cache.front();
      g_cache.erase(g_cache.begin());
    }
    g_cache.push_back(e);
  }
  if (flags & QFT_BATCH_EAGER) {
    he = launch_entry(e, (hipStream_t)stream);
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

}  // extern "C"
