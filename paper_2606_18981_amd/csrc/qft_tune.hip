// Autotuner and tuning cache; see include/qft_tune.h.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qft.h"
#include "../../include/qft_tune.h"
#include "qft_planner.h"
#include "qft_runtime.h"

using namespace qft;

namespace {

using Key = std::tuple<int, int, int>;  // n, effective cutoff, layout (dtype | order)

struct Entry {
  qft_config_t cfg;
  double ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_table;

Key make_key(int n, int cutoff, int layout) {
  const int keff = (cutoff < 0 || cutoff >= n - 1) ? n - 1 : cutoff;
  return Key(n, keff, layout & (QFT_C128 | QFT_ORDER_BITREV));
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "gfx950";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Candidates: tile 2^t elements, register radix 2^r (the qubits fused per
// register group, the paper's fusion width), spectator widths c and b.
// Radix 64 (six fused qubits) would hold 128 complex64 data registers per
// lane, more than two waves per SIMD allow; the kernels stop at radix 32.
std::vector<qft_config_t> candidate_grid(int tmin = 8, int tmax = 14, int cmax = 5) {
  std::vector<qft_config_t> v;
  for (int t = tmin; t <= tmax; ++t)
    for (int r = 3; r <= 5; ++r)
      for (int c = 2; c <= cmax; ++c)
        for (int b = 2; b <= 4; ++b) {
          qft_config_t q;
          memset(&q, 0, sizeof(q));
          q.tile_log2 = t;
          q.radix_log2 = r;
          q.spec_log2 = c;
          q.rev_spec_log2 = b;
          v.push_back(q);
        }
  return v;
}

// identity of the launches a configuration produces (to skip duplicates)
std::string plan_signature(const HostPlan &hp) {
  std::string s;
  char buf[96];
  for (const PassLaunch &L : hp.passes) {
    snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%d;", L.d.lo, L.d.m, L.d.pbase, L.d.r, L.d.T,
             L.threads);
    s += buf;
  }
  return s;
}

// unique candidate configurations for one shape
std::vector<qft_config_t> unique_candidates(int n, int cutoff, int norm, int layout) {
  std::vector<qft_config_t> out;
  std::set<std::string> seen;
  for (const qft_config_t &c : candidate_grid()) {
    HostPlan hp;
    std::string err;
    if (build_host_plan(n, cutoff, norm, layout, &c, hp, err) != QFT_OK) continue;
    if (seen.insert(plan_signature(hp)).second) out.push_back(c);
  }
  return out;
}

bool get_num(const char *line, const char *key, double *v) {
  char pat[64];
  snprintf(pat, sizeof pat, "\"%s\":", key);
  const char *p = strstr(line, pat);
  if (!p) return false;
  p += strlen(pat);
  char *end = nullptr;
  *v = strtod(p, &end);
  return end != p;
}

bool get_str(const char *line, const char *key, std::string *v) {
  char pat[64];
  snprintf(pat, sizeof pat, "\"%s\":\"", key);
  const char *p = strstr(line, pat);
  if (!p) return false;
  p += strlen(pat);
  const char *q = strchr(p, '"');
  if (!q) return false;
  v->assign(p, q - p);
  return true;
}

// The tuner's stream and its two timing events; on failure nothing stays
// allocated.
int tuner_resources(hipStream_t *s, hipEvent_t *a, hipEvent_t *b) {
  hipError_t he = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
  if (he != hipSuccess) return hip_error(he, "tuner stream");
  if ((he = hipEventCreate(a)) != hipSuccess) {
    (void)hipStreamDestroy(*s);
    return hip_error(he, "tuner events");
  }
  if ((he = hipEventCreate(b)) != hipSuccess) {
    (void)hipEventDestroy(*a);
    (void)hipStreamDestroy(*s);
    return hip_error(he, "tuner events");
  }
  return QFT_OK;
}

int time_plan(qft_plan_t *p, void *data, int reps, hipStream_t s, hipEvent_t a, hipEvent_t b,
              double *ms) {
  int rc = qft_execute(p, data, s);
  if (rc != QFT_OK) return rc;
  hipError_t he = hipEventRecord(a, s);
  if (he != hipSuccess) return hip_error(he, "tuner timing");
  for (int i = 0; i < reps; ++i) {
    rc = qft_execute(p, data, s);
    if (rc != QFT_OK) return rc;
  }
  if ((he = hipEventRecord(b, s)) != hipSuccess) return hip_error(he, "tuner timing");
  if ((he = hipEventSynchronize(b)) != hipSuccess) return hip_error(he, "tuner timing");
  float f = 0.f;
  if ((he = hipEventElapsedTime(&f, a, b)) != hipSuccess) return hip_error(he, "tuner timing");
  *ms = f / reps;
  return QFT_OK;
}

}  // namespace

namespace qft {
bool tune_table_lookup(int n, int cutoff, int layout, qft_config_t *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(make_key(n, cutoff, layout));
  if (it == g_table.end()) return false;
  *out = it->second.cfg;
  return true;
}
}  // namespace qft

extern "C" {

int qft_tune_lookup(int n, int cutoff, int layout, qft_config_t *out) {
  clear_error();
  if (!out) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!tune_table_lookup(n, cutoff, layout, out))
    return set_error(QFT_ERR_INVALID, "no tuning entry for this shape");
  return QFT_OK;
}

int qft_tune_insert(int n, int cutoff, int layout, const qft_config_t *config, double ms) {
  clear_error();
  if (!config) return set_error(QFT_ERR_INVALID, "NULL argument");
  HostPlan hp;
  std::string err;
  int rc = build_host_plan(n, cutoff, QFT_NORM_UNITARY, layout & ~QFT_SCHEDULE_GATES, config, hp,
                           err);
  if (rc != QFT_OK) return set_error(rc, err);
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[make_key(n, cutoff, layout)] = Entry{*config, ms};
  return QFT_OK;
}

int qft_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  return QFT_OK;
}

int qft_tune(int n, int cutoff, int norm, int layout, void *data, int reps, qft_config_t *best,
             double *best_ms) {
  clear_error();
  if (!data) return set_error(QFT_ERR_POINTER, "data pointer is NULL");
  if (reps < 1) return set_error(QFT_ERR_INVALID, "reps must be >= 1");
  if (layout & QFT_SCHEDULE_GATES)
    return set_error(QFT_ERR_UNSUPPORTED, "only the fused schedule is tuned");
  std::vector<qft_config_t> cands = unique_candidates(n, cutoff, norm, layout);
  if (cands.empty()) return set_error(QFT_ERR_UNSUPPORTED, "no valid configuration");
  hipStream_t s;
  hipEvent_t a, b;
  {
    const int r = tuner_resources(&s, &a, &b);
    if (r != QFT_OK) return r;
  }
  double bms = 1e300;
  qft_config_t bc = cands[0];
  int rc = QFT_OK;
  for (const qft_config_t &c : cands) {
    qft_plan_t *p = qft_plan_config(n, cutoff, norm, layout, &c);
    if (!p) {
      rc = QFT_ERR_INVALID;
      break;
    }
    double ms = 0;
    rc = time_plan(p, data, reps, s, a, b, &ms);
    qft_destroy(p);
    if (rc != QFT_OK) break;
    if (ms < bms) {
      bms = ms;
      bc = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  if (rc != QFT_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[make_key(n, cutoff, layout)] = Entry{bc, bms};
  }
  if (best) *best = bc;
  if (best_ms) *best_ms = bms;
  return QFT_OK;
}

int qft_tune_batch(const int *n, const int *cutoff, int count, int norm, int layout,
                   void *const *data, int reps, qft_config_t *best, double *best_ms) {
  clear_error();
  if (count < 1 || !n || !cutoff || !data || reps < 1)
    return set_error(QFT_ERR_INVALID, "invalid batch tuning arguments");
  hipStream_t s;
  hipEvent_t a, b;
  {
    const int r = tuner_resources(&s, &a, &b);
    if (r != QFT_OK) return r;
  }
  hipError_t he = hipSuccess;
  double bms = 1e300;
  qft_config_t bc{};
  bool found = false;
  int rc = QFT_OK;
  // the batch grid: tiles of 2^8..2^14 elements (the batch's transforms have
  // 2^8..2^20; 2^14 complex64 tiles run the four-wave kernels), radix 8..32,
  // spectator widths 2..4
  for (const qft_config_t &c : candidate_grid(8, 14, 4)) {
    // one plan per distinct shape, shared by the transforms of that shape
    std::map<std::pair<int, int>, qft_plan_t *> plans;
    std::vector<qft_plan_t *> pv(count, nullptr);
    bool ok = true;
    for (int i = 0; i < count && ok; ++i) {
      auto k = std::make_pair(n[i], cutoff[i]);
      auto it = plans.find(k);
      if (it == plans.end()) {
        qft_plan_t *p = qft_plan_config(n[i], cutoff[i], norm, layout, &c);
        if (!p) {
          ok = false;
          break;
        }
        it = plans.emplace(k, p).first;
      }
      pv[i] = it->second;
    }
    if (ok) {
      // the first call builds the work list and captures the graph
      int r1 = qft_execute_batch_ex(pv.data(), data, count, 0, s);
      if (r1 == QFT_OK) {
        he = hipEventRecord(a, s);
        for (int i = 0; i < reps && r1 == QFT_OK && he == hipSuccess; ++i)
          r1 = qft_execute_batch_ex(pv.data(), data, count, 0, s);
        if (he == hipSuccess) he = hipEventRecord(b, s);
        if (he == hipSuccess) he = hipEventSynchronize(b);
        float f = 0.f;
        if (he == hipSuccess && r1 == QFT_OK) he = hipEventElapsedTime(&f, a, b);
        if (he != hipSuccess) {
          rc = hip_error(he, "batch tuner timing");
        } else if (r1 == QFT_OK) {
          const double ms = f / reps;
          if (ms < bms) {
            bms = ms;
            bc = c;
            found = true;
          }
        }
      }
    }
    for (auto &kv : plans) qft_destroy(kv.second);
    if (rc != QFT_OK) break;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  if (rc != QFT_OK) return rc;
  if (!found) return set_error(QFT_ERR_UNSUPPORTED, "no configuration ran the batch");
  // (the per-shape table is left alone: the batch's winner is best for the
  // batch as a whole, not for each shape alone)
  if (best) *best = bc;
  if (best_ms) *best_ms = bms;
  return QFT_OK;
}

int qft_tune_save(const char *path) {
  clear_error();
  if (!path) return set_error(QFT_ERR_INVALID, "NULL path");
  FILE *f = fopen(path, "w");
  if (!f) return set_error(QFT_ERR_INVALID, std::string("cannot write ") + path);
  const std::string arch = arch_name();
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto &kv : g_table) {
    const Entry &e = kv.second;
    std::string split, tiles;
    for (int i = 0; i < QFT_MAX_PASSES && e.cfg.pass_bits[i] > 0; ++i)
      split += (i ? "," : "") + std::to_string(e.cfg.pass_bits[i]);
    for (int i = 0; i < QFT_MAX_PASSES; ++i)
      tiles += (i ? "," : "") + std::to_string(e.cfg.pass_tile_log2[i]);
    fprintf(f,
            "{\"arch\":\"%s\",\"n\":%d,\"cutoff\":%d,\"layout\":%d,\"tile_log2\":%d,"
            "\"radix_log2\":%d,\"spec_log2\":%d,\"rev_spec_log2\":%d,\"nontemporal\":%d,"
            "\"pass_bits\":\"%s\",\"pass_tile_log2\":\"%s\",\"ms\":%.6g}\n",
            arch.c_str(), std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
            e.cfg.tile_log2, e.cfg.radix_log2, e.cfg.spec_log2, e.cfg.rev_spec_log2,
            e.cfg.nontemporal, split.c_str(), tiles.c_str(), e.ms);
  }
  fclose(f);
  return QFT_OK;
}

int qft_tune_load(const char *path) {
  clear_error();
  if (!path) return set_error(QFT_ERR_INVALID, "NULL path");
  FILE *f = fopen(path, "r");
  if (!f) return set_error(QFT_ERR_INVALID, std::string("cannot read ") + path);
  const std::string arch = arch_name();
  char line[1024];
  int count = 0;
  while (fgets(line, sizeof line, f)) {
    std::string a;
    double n, k, lay, t, r, c, b, ms;
    if (!get_str(line, "arch", &a) || a != arch) continue;
    if (!get_num(line, "n", &n) || !get_num(line, "cutoff", &k) ||
        !get_num(line, "layout", &lay) || !get_num(line, "tile_log2", &t) ||
        !get_num(line, "radix_log2", &r) || !get_num(line, "spec_log2", &c) ||
        !get_num(line, "rev_spec_log2", &b))
      continue;
    if (!get_num(line, "ms", &ms)) ms = 0.0;
    qft_config_t cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.tile_log2 = (int)t;
    cfg.radix_log2 = (int)r;
    cfg.spec_log2 = (int)c;
    cfg.rev_spec_log2 = (int)b;
    double ntv;
    if (get_num(line, "nontemporal", &ntv)) cfg.nontemporal = (int)ntv;
    std::string split;
    if (get_str(line, "pass_bits", &split) && !split.empty()) {
      const char *q = split.c_str();
      for (int i = 0; i < QFT_MAX_PASSES && *q; ++i) {
        char *end = nullptr;
        cfg.pass_bits[i] = (int)strtol(q, &end, 10);
        if (end == q) break;
        q = *end == ',' ? end + 1 : end;
      }
    }
    std::string tiles;
    if (get_str(line, "pass_tile_log2", &tiles) && !tiles.empty()) {
      const char *q = tiles.c_str();
      for (int i = 0; i < QFT_MAX_PASSES && *q; ++i) {
        char *end = nullptr;
        cfg.pass_tile_log2[i] = (int)strtol(q, &end, 10);
        if (end == q) break;
        q = *end == ',' ? end + 1 : end;
      }
    }
    // an entry the planner rejects is skipped
    HostPlan hp;
    std::string err;
    if (build_host_plan((int)n, (int)k, QFT_NORM_UNITARY, (int)lay, &cfg, hp, err) != QFT_OK)
      continue;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[make_key((int)n, (int)k, (int)lay)] = Entry{cfg, ms};
    ++count;
  }
  fclose(f);
  return count;
}

}  // extern "C"
