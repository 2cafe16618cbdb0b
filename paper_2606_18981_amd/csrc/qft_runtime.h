// Runtime-side plan object and helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/qft.h"
#include "qft_internal.h"
#include "qft_planner.h"

namespace qft {

// Event pairs around every launch of timed executes.
struct LaunchTimer {
  std::vector<hipEvent_t> events;
  long long execs = 0;
  size_t cur_base = 0;
  int nl = 0;
  hipEvent_t slot(size_t i);
  hipError_t begin(int launches);  // creates the events it needs
  void end();
  void release();
};

int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
void clear_error();

}  // namespace qft

struct qft_plan_s {
  qft::HostPlan hp;
  int device = 0;
  void *d_tables = nullptr;
  void *d_ws = nullptr;
  double *d_norm = nullptr;  // partial sums for qft_execute_norm (lazy)
  uint32_t norm_parts = 0;
  std::vector<qft::PassLaunch> launches;  // table pointers resolved
  bool timing = false;
  qft::LaunchTimer timer;
  int num_launches() const {
    if (hp.schedule == qft::Schedule::Fused) return (int)launches.size();
    return (int)hp.gates.size() + (hp.gate_norm != 1.0 ? 1 : 0);
  }
};

namespace qft {
// The last pass of an execute that also compares its output with a
// reference output `ref` (same layout), writing `part`: the per-wave
// comparison partials (kCmpSlots doubles each) of that pass's tiles.
struct FusedCompare {
  const void *ref;
  double *part;
};
// norm_out: device double receiving ||x||_2 of the input, or nullptr; part:
// device buffer of norm_parts_for(p) partial sums (used when norm_out is set);
// allow_timing: record the plan's per-launch timing events if it has them on;
// cmp: compare in the last pass (fused schedule), or nullptr
int enqueue_plan(qft_plan_s *p, void *dev, void *ws, hipStream_t s, double *norm_out,
                 double *part, bool allow_timing, const FusedCompare *cmp = nullptr);
// partial sums of |x|^2 an execute with the input norm needs for this plan
uint32_t norm_parts_for(const qft_plan_s *p);
// argument checks shared by the execute entry points (no device work)
int check_execute(qft_plan_s *plan, void *dev_ptr, void *workspace);
// drop cached batch launches that use this plan
void batch_forget_plan(qft_plan_s *plan);
// tuned configuration for a plan shape, if the tuning table has one
bool tune_table_lookup(int n, int cutoff, int layout, qft_config_t *out);
}
