// Host planner: gate list, pass partition, register/thread maps and FP64
// twiddle tables.  Pure C++ (no device calls), so it can run without a GPU.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/qft.h"
#include "qft_internal.h"

namespace qft {

enum class Schedule { Fused, Gates };

struct Gate {
  int kind;      // 0 = H, 1 = controlled phase, 2 = swap
  int a, b;      // H: target a; CR: control a, target b; SWAP: qubits a, b
  int m;         // CR: R_m
  double re, im; // CR: exp(-2 pi i / 2^m) in FP64
};

struct HostPlan {
  int n = 0;
  int keff = 0;        // effective cutoff
  int norm = 0;
  int layout = 0;
  bool c128 = false;
  bool bitrev = false;
  bool inverse = false; // conjugate-phase circuit (QFT_INVERSE)
  Schedule schedule = Schedule::Fused;
  qft_config_t cfg{};  // resolved configuration
  bool auto_radix = true;  // radix_log2 not given: the planner may pick it
  size_t elem_bytes = 0;
  size_t state_bytes = 0;
  size_t ws_bytes = 0;
  long long gates_h = 0, gates_cr = 0, gates_swap = 0;

  // fused schedule
  std::vector<PassLaunch> passes;
  int MI = 1;          // internal table exponent
  int L = 0;           // two-level table split
  bool need_ext = false;
  // table image (in the plan's dtype), byte offsets of each table
  std::vector<unsigned char> tables;
  size_t off_int = 0, off_lo = 0, off_hi = 0;
  // per pass: byte offset of its per-thread group-0 factor table, or 0 (none)
  std::vector<size_t> off_gtab;
  // per pass: the same for group 1 (three-group passes), or 0
  std::vector<size_t> off_gtab1;
  size_t end_hi = 0;  // end of the high table (the group tables follow)

  // gate schedule
  std::vector<Gate> gates;
  double gate_norm = 1.0;  // final scale for norm != unitary

  size_t hbm_bytes() const;
};

// Build the host plan.  Returns QFT_OK or an error code with `err` set.
int build_host_plan(int n, int cutoff, int norm, int layout,
                    const qft_config_t *cfg, HostPlan &out, std::string &err);

// Fill a qft_plan_info from a host plan.
void describe_plan(const HostPlan &p, qft_plan_info_t *out);

// w_N^m = exp(-2 pi i m / N) for N = 2^logN, from the exact dyadic angle
// m / N reduced to the first octant (long-double cos/sin, rounded once).
void omega_pow2(int logN, uint64_t m, double *re, double *im);

// Default kernel configuration for a dtype.
qft_config_t default_config(bool c128);

}  // namespace qft
