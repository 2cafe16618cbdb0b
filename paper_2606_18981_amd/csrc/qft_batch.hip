// Batched uneven-size execution (persistent kernel); see include/qft.h.
#include <hip/hip_runtime.h>

#include "../../include/qft.h"
#include "qft_runtime.h"

using namespace qft;

extern "C" int qft_execute_batch(qft_plan_t *const *plans, void *const *dev_ptrs, int count,
                                 qft_stream_t stream) {
  clear_error();
  (void)plans;
  (void)dev_ptrs;
  (void)count;
  (void)stream;
  return set_error(QFT_ERR_UNSUPPORTED, "batched execution is not built yet");
}
