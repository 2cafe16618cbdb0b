// Host-only driver for tests/test_planner_asan_cpu.py: builds and describes
// plans over every size, layout and norm, a spread of cutoffs and a grid of
// kernel configurations, with the planner compiled under AddressSanitizer
// and UndefinedBehaviorSanitizer.  Prints the accepted and rejected counts.
#include <cstdio>
#include <string>

#include "qft_planner.h"

using namespace qft;

int main() {
  long ok = 0, rejected = 0;
  auto one = [&](int n, int k, int norm, int layout, const qft_config_t *cfg) {
    HostPlan hp;
    std::string err;
    if (build_host_plan(n, k, norm, layout, cfg, hp, err) == 0) {
      qft_plan_info_t info;
      describe_plan(hp, &info);
      ++ok;
    } else {
      ++rejected;
    }
  };
  const int layouts[] = {0, 1, 2, 3, 4, 5, 0x10, 0x11, 0x12, 0x13, 0x40};
  for (int n = -1; n <= 33; ++n)
    for (int layout : layouts)
      for (int k : {-2, -1, 0, 1, 3, n / 2, n - 2, n - 1, n, n + 5})
        for (int norm = -1; norm < 4; ++norm) one(n, k, norm, layout, nullptr);
  for (int T = 0; T <= 16; ++T)
    for (int r = 0; r <= 6; ++r)
      for (int sp = -1; sp <= 6; ++sp)
        for (int n : {1, 5, 12, 17, 21, 24, 28, 30}) {
          qft_config_t c = {};
          c.tile_log2 = T;
          c.radix_log2 = r;
          c.spec_log2 = sp;
          c.rev_spec_log2 = sp;
          for (int layout : {0, 1, 2}) one(n, n > 8 ? 6 : -1, 0, layout, &c);
        }
  printf("ok %ld rejected %ld\n", ok, rejected);
  return 0;
}
