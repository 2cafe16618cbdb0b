// Planner introspection for tests; see include/qft_debug.h.  Host only.
#include "../../include/qft_debug.h"

#include <string.h>

#include <string>

#include "qft_planner.h"

using namespace qft;

extern "C" {

size_t qft_debug_pass_desc_size(void) { return sizeof(PassDesc); }

int qft_debug_pass(int n, int cutoff, int norm, int layout, const qft_config_t *config, int pass,
                   void *out_desc, size_t desc_bytes, int *launch) {
  HostPlan hp;
  std::string err;
  int rc = build_host_plan(n, cutoff, norm, layout, config, hp, err);
  if (rc != QFT_OK) return rc;
  if (hp.schedule != Schedule::Fused) return QFT_ERR_UNSUPPORTED;
  if (pass < 0 || pass >= (int)hp.passes.size()) return QFT_ERR_INVALID;
  if (!out_desc || desc_bytes < sizeof(PassDesc)) return QFT_ERR_INVALID;
  PassLaunch L = hp.passes[pass];
  L.d.tw_int = L.d.tw_lo = L.d.tw_hi = nullptr;
  // the group-factor tables: their byte offsets in the table image (0: none)
  L.d.gtab = reinterpret_cast<const void *>((uintptr_t)hp.off_gtab[pass]);
  L.d.gtab1 = reinterpret_cast<const void *>((uintptr_t)hp.off_gtab1[pass]);
  memcpy(out_desc, &L.d, sizeof(PassDesc));
  if (launch) {
    launch[0] = L.threads;
    launch[1] = L.lds_bytes;
    launch[2] = (int)L.grid;
    launch[3] = L.in_ws;
    launch[4] = L.out_ws;
  }
  return QFT_OK;
}

int qft_debug_tables(int n, int cutoff, int norm, int layout, const qft_config_t *config,
                     void *out, size_t out_bytes, size_t *offsets) {
  HostPlan hp;
  std::string err;
  int rc = build_host_plan(n, cutoff, norm, layout, config, hp, err);
  if (rc != QFT_OK) return rc;
  if (offsets) {
    offsets[0] = hp.off_int;
    offsets[1] = hp.off_lo;
    offsets[2] = hp.off_hi;
    offsets[3] = hp.end_hi;
    offsets[4] = hp.tables.size();
  }
  if (out) {
    if (out_bytes < hp.tables.size()) return QFT_ERR_INVALID;
    memcpy(out, hp.tables.data(), hp.tables.size());
  }
  return QFT_OK;
}

}  // extern "C"
