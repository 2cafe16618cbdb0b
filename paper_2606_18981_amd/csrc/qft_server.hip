// Continuous-batching request server on one GPU; see include/qft_serve.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/qft.h"
#include "../../include/qft_serve.h"
#include "qft_kernels.h"
#include "qft_runtime.h"
#include "qft_sched.h"

using namespace qft;

namespace {

using PlanKey = std::tuple<int, int, int, int>;  // n, effective cutoff, norm, layout

// Size-bucketed device memory cache: freed blocks are kept for reuse, so the
// steady state makes no hipMalloc / hipFree calls.
struct BlockPool {
  std::map<size_t, std::vector<void *>> free_blocks;
  std::vector<void *> all;
  void *get(size_t bytes, hipError_t *err) {
    auto it = free_blocks.find(bytes);
    if (it != free_blocks.end() && !it->second.empty()) {
      void *p = it->second.back();
      it->second.pop_back();
      *err = hipSuccess;
      return p;
    }
    void *p = nullptr;
    *err = hipMalloc(&p, bytes);
    if (*err != hipSuccess) {
      // give cached blocks of other sizes back and retry once (the retry
      // reports any device error)
      (void)hipDeviceSynchronize();
      for (auto &kv : free_blocks)
        for (void *q : kv.second) {
          (void)hipFree(q);
          all.erase(std::find(all.begin(), all.end(), q));
        }
      free_blocks.clear();
      *err = hipMalloc(&p, bytes);
      if (*err != hipSuccess) return nullptr;
    }
    all.push_back(p);
    return p;
  }
  void put(void *p, size_t bytes) {
    if (p) free_blocks[bytes].push_back(p);
  }
  void clear() {
    for (void *p : all) (void)hipFree(p);
    all.clear();
    free_blocks.clear();
  }
};

}  // namespace

struct qft_server_s {
  size_t budget = 0;
  int max_inflight = 1;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::map<PlanKey, qft_plan_t *> plans;
  BlockPool pool;
  ~qft_server_s() {
    for (auto &kv : plans) qft_destroy(kv.second);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    pool.clear();
  }
  PlanKey key(const qft_request_t &r) const {
    const int keff = (r.cutoff < 0 || r.cutoff >= r.n - 1) ? -1 : r.cutoff;
    return PlanKey(r.n, keff, r.norm, r.layout);
  }
};

namespace {

struct GpuDevice {
  qft_server_s *srv;
  const qft_request_t *reqs;
  std::vector<qft_request_result_t> *res;
  std::chrono::steady_clock::time_point t0;
  struct Slot {
    void *state = nullptr, *ws = nullptr;
    size_t state_bytes = 0, ws_bytes = 0;
    hipEvent_t ev = nullptr;
    int stream = -1;
  };
  std::vector<Slot> slots;
  std::vector<hipEvent_t> free_events;
  std::vector<int> stream_load;
  double hbm_bytes = 0.0;

  double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  int start(int r) {
    const qft_request_t &q = reqs[r];
    auto it = srv->plans.find(srv->key(q));
    if (it == srv->plans.end()) return set_error(QFT_ERR_INVALID, "request plan not prepared");
    qft_plan_t *p = it->second;
    Slot &s = slots[r];
    hipError_t he;
    s.state_bytes = p->hp.state_bytes;
    s.state = srv->pool.get(s.state_bytes, &he);
    if (!s.state) return hip_error(he, "request state allocation");
    s.ws_bytes = p->hp.ws_bytes;
    if (s.ws_bytes) {
      s.ws = srv->pool.get(s.ws_bytes, &he);
      if (!s.ws) return hip_error(he, "request workspace allocation");
    }
    // least-loaded stream of the pool
    int best = 0;
    for (int i = 1; i < (int)srv->streams.size(); ++i)
      if (stream_load[i] < stream_load[best]) best = i;
    hipStream_t st = srv->streams[best];
    int rc = enqueue(q, p, s, st);
    if (rc != QFT_OK) {
      // part of the request may be on the stream: let it finish before
      // release() hands the slot's memory to another request
      (void)hipStreamSynchronize(st);
      return rc;
    }
    s.stream = best;
    ++stream_load[best];
    (*res)[r].stream = best;
    hbm_bytes += (double)p->hp.hbm_bytes() + (double)s.state_bytes;  // + input write
    return QFT_OK;
  }
  // input generation, transform, optional result copy and completion event
  int enqueue(const qft_request_t &q, qft_plan_t *p, Slot &s, hipStream_t st) {
    int rc = qft_fill_random(s.state, q.n, q.layout, q.dist, q.seed, 0, st);
    if (rc != QFT_OK) return rc;
    rc = qft_execute_ws(p, s.state, s.ws, st);
    if (rc != QFT_OK) return rc;
    hipError_t he;
    if (q.out) {
      he = hipMemcpyAsync(q.out, s.state, s.state_bytes, hipMemcpyDeviceToDevice, st);
      if (he != hipSuccess) return hip_error(he, "result copy");
    }
    if (free_events.empty()) {
      hipEvent_t ev;
      he = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (he != hipSuccess) return hip_error(he, "event create");
      free_events.push_back(ev);
    }
    s.ev = free_events.back();
    free_events.pop_back();
    he = hipEventRecord(s.ev, st);
    if (he != hipSuccess) return hip_error(he, "event record");
    return QFT_OK;
  }
  bool poll(int r, int *status) {
    Slot &s = slots[r];
    hipError_t he = hipEventQuery(s.ev);
    if (he == hipErrorNotReady) return false;
    *status = he == hipSuccess ? QFT_OK : QFT_ERR_HIP;
    return true;
  }
  void release(int r) {
    Slot &s = slots[r];
    srv->pool.put(s.state, s.state_bytes);
    srv->pool.put(s.ws, s.ws_bytes);
    if (s.ev) free_events.push_back(s.ev);
    if (s.stream >= 0) --stream_load[s.stream];
    s = Slot();
  }
  void idle(double next_arrival) {
    const double t = now();
    bool any_inflight = false;
    for (int l : stream_load) any_inflight |= l > 0;
    if (!any_inflight && next_arrival > t + 200e-6) {
      std::this_thread::sleep_for(std::chrono::duration<double>(next_arrival - t - 100e-6));
    } else {
      std::this_thread::yield();
    }
  }
};

}  // namespace

extern "C" {

qft_server_t *qft_server_create(size_t hbm_budget_bytes, int max_inflight, int num_streams) {
  clear_error();
  if (max_inflight < 1 || num_streams < 1 || hbm_budget_bytes == 0) {
    set_error(QFT_ERR_INVALID, "budget, slots and streams must be positive");
    return nullptr;
  }
  qft_server_s *s = new (std::nothrow) qft_server_s();
  if (!s) return nullptr;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    set_error(QFT_ERR_HIP, "hipGetDevice failed");
    return nullptr;
  }
  for (int i = 0; i < num_streams; ++i) {
    hipStream_t st;
    hipError_t he = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (he != hipSuccess) {
      hip_error(he, "stream create");
      delete s;
      return nullptr;
    }
    s->streams.push_back(st);
  }
  return s;
}

void qft_server_destroy(qft_server_t *server) {
  if (!server) return;
  (void)hipDeviceSynchronize();  // nothing of the server may still run
  delete server;
}

int qft_server_prepare(qft_server_t *server, const qft_request_t *reqs, int count) {
  clear_error();
  if (!server || (count > 0 && !reqs)) return set_error(QFT_ERR_INVALID, "NULL argument");
  for (int i = 0; i < count; ++i) {
    const qft_request_t &r = reqs[i];
    if (r.layout & QFT_SCHEDULE_GATES)
      return set_error(QFT_ERR_UNSUPPORTED, "the server runs fused-schedule plans");
    PlanKey k = server->key(r);
    if (server->plans.count(k)) continue;
    // requests bring their own workspace from the server's pool
    qft_plan_t *p = qft_plan(r.n, r.cutoff, r.norm, r.layout | QFT_PLAN_NO_WORKSPACE);
    if (!p) return QFT_ERR_INVALID;
    server->plans[k] = p;
  }
  return QFT_OK;
}

int qft_server_run(qft_server_t *server, const qft_request_t *reqs, int count,
                   qft_request_result_t *results, qft_server_stats_t *stats) {
  clear_error();
  if (!server || count < 0 || (count > 0 && (!reqs || !results)))
    return set_error(QFT_ERR_INVALID, "NULL argument");
  for (int i = 1; i < count; ++i)
    if (reqs[i].arrival < reqs[i - 1].arrival)
      return set_error(QFT_ERR_INVALID, "requests must be sorted by arrival");
  int rc = qft_server_prepare(server, reqs, count);
  if (rc != QFT_OK) return rc;
  // the resident plans' device memory (tables) is charged once, up front
  size_t plan_bytes = 0;
  for (const auto &kv : server->plans) plan_bytes += qft_plan_device_bytes(kv.second);
  if (plan_bytes >= server->budget)
    return set_error(QFT_ERR_NOMEM, "the resident plans alone exceed the HBM budget");
  std::vector<SchedReq> sr(count);
  for (int i = 0; i < count; ++i) {
    const qft_plan_t *p = server->plans[server->key(reqs[i])];
    sr[i].arrival = reqs[i].arrival;
    sr[i].bytes = p->hp.state_bytes + p->hp.ws_bytes;
  }
  std::vector<qft_request_result_t> res;
  GpuDevice dev;
  dev.srv = server;
  dev.reqs = reqs;
  dev.res = &res;
  dev.slots.resize(count);
  dev.stream_load.assign(server->streams.size(), 0);
  qft_server_stats_t st;
  res.assign(count, qft_request_result_t{});
  dev.t0 = std::chrono::steady_clock::now();
  run_schedule(dev, sr, server->budget - plan_bytes, server->max_inflight, res, st);
  st.hbm_bytes = dev.hbm_bytes;
  st.plan_bytes = plan_bytes;
  st.peak_reserved_bytes += plan_bytes;
  for (hipEvent_t ev : dev.free_events) (void)hipEventDestroy(ev);
  for (int i = 0; i < count; ++i) results[i] = res[i];
  if (stats) *stats = st;
  return st.failed ? QFT_ERR_HIP : QFT_OK;
}

int qft_server_simulate(size_t hbm_budget_bytes, int max_inflight, const double *arrival,
                        const size_t *bytes, const double *service, int count,
                        qft_request_result_t *results, qft_server_stats_t *stats) {
  clear_error();
  if (max_inflight < 1 || count < 0 || (count > 0 && (!arrival || !bytes || !service || !results)))
    return set_error(QFT_ERR_INVALID, "invalid arguments");
  std::vector<SchedReq> sr(count);
  std::vector<double> sv(service, service + count);
  for (int i = 0; i < count; ++i) {
    if (i > 0 && arrival[i] < arrival[i - 1])
      return set_error(QFT_ERR_INVALID, "requests must be sorted by arrival");
    sr[i].arrival = arrival[i];
    sr[i].bytes = bytes[i];
  }
  SimDevice dev(sv);
  std::vector<qft_request_result_t> res;
  qft_server_stats_t st;
  run_schedule(dev, sr, hbm_budget_bytes, max_inflight, res, st);
  for (int i = 0; i < count; ++i) results[i] = res[i];
  if (stats) *stats = st;
  return QFT_OK;
}

}  // extern "C"
