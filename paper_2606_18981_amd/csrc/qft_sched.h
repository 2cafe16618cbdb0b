// Scheduler core of the request server, independent of the device so that
// the same admission logic runs on the GPU and in a simulated test device.
//
// Dev must provide:
//   double now();                       seconds since the start of the run
//   int start(int r);                   enqueue request r, QFT_OK or error
//   bool poll(int r, int *status);      true once request r has finished
//   void release(int r);                return r's memory
//   void idle(double next_arrival);     nothing to do: wait a little
#pragma once
#include <stddef.h>

#include <algorithm>
#include <deque>
#include <vector>

#include "../../include/qft.h"
#include "../../include/qft_serve.h"

namespace qft {

struct SchedReq {
  double arrival;
  size_t bytes;
};

template <class Dev>
void run_schedule(Dev &dev, const std::vector<SchedReq> &reqs, size_t budget, int max_inflight,
                  std::vector<qft_request_result_t> &res, qft_server_stats_t &st) {
  const size_t count = reqs.size();
  res.assign(count, qft_request_result_t{});
  st = qft_server_stats_t{};
  std::deque<int> pending;
  std::vector<int> inflight;
  size_t reserved = 0, next = 0, done = 0;
  for (size_t i = 0; i < count; ++i) {
    res[i].arrival = reqs[i].arrival;
    res[i].bytes = reqs[i].bytes;
    res[i].stream = -1;
  }
  while (done < count) {
    bool progress = false;
    double now = dev.now();
    while (next < count && reqs[next].arrival <= now) pending.push_back((int)next++);
    // completions free budget and slots
    for (size_t i = 0; i < inflight.size();) {
      const int r = inflight[i];
      int status = QFT_OK;
      if (dev.poll(r, &status)) {
        res[r].completed = dev.now();
        res[r].status = status;
        if (status == QFT_OK) ++st.completed;
        else ++st.failed;
        reserved -= reqs[r].bytes;
        dev.release(r);
        inflight.erase(inflight.begin() + i);
        ++done;
        progress = true;
      } else {
        ++i;
      }
    }
    // FIFO admission: the head waits until both a slot and its bytes are free
    now = dev.now();
    while (!pending.empty()) {
      const int r = pending.front();
      if (reqs[r].bytes > budget) {  // can never be admitted
        res[r].admitted = res[r].completed = now;
        res[r].status = QFT_ERR_BUSY;
        ++st.failed;
        pending.pop_front();
        ++done;
        progress = true;
        continue;
      }
      if ((int)inflight.size() >= max_inflight || reserved + reqs[r].bytes > budget) break;
      res[r].admitted = now;
      const int status = dev.start(r);
      pending.pop_front();
      progress = true;
      if (status != QFT_OK) {
        res[r].completed = now;
        res[r].status = status;
        ++st.failed;
        dev.release(r);
        ++done;
        continue;
      }
      reserved += reqs[r].bytes;
      inflight.push_back(r);
      st.peak_reserved_bytes = std::max(st.peak_reserved_bytes, reserved);
      st.peak_inflight = std::max(st.peak_inflight, (int)inflight.size());
    }
    if (!progress && done < count) dev.idle(next < count ? reqs[next].arrival : -1.0);
  }
  st.wall_seconds = dev.now();
}

// Simulated device: virtual clock, request r finishes service[r] seconds
// after it is started.
struct SimDevice {
  const std::vector<double> &service;
  std::vector<double> finish;
  double t = 0.0;
  explicit SimDevice(const std::vector<double> &s) : service(s), finish(s.size(), 0.0) {}
  double now() { return t; }
  int start(int r) {
    finish[r] = t + service[r];
    return QFT_OK;
  }
  bool poll(int r, int *status) {
    *status = QFT_OK;
    return finish[r] <= t;
  }
  void release(int) {}
  void idle(double next_arrival) {
    // jump to the next event: an arrival or the earliest unfinished finish
    double nxt = next_arrival >= 0 ? next_arrival : 1e300;
    for (double f : finish)
      if (f > t) nxt = std::min(nxt, f);
    t = nxt < 1e300 ? nxt : t;
  }
};

}  // namespace qft
