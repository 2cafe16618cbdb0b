/*
 * qft_debug.h - planner introspection for tests (libqft.so).
 *
 * These calls run the host planner only (no device use) and copy out its
 * internal launch descriptors, so that tests can check the pass partition,
 * the register/thread maps and the twiddle tables on a machine without a GPU.
 * The descriptor layout is internal and may change with the library.
 */
#ifndef QFT_MI355X_DEBUG_H
#define QFT_MI355X_DEBUG_H

#include <stddef.h>

#include "qft.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size in bytes of one internal pass descriptor (struct qft::PassDesc).    */
size_t qft_debug_pass_desc_size(void);

/* Copy the descriptor of launch `pass` of the plan qft_plan_config would
 * build into out_desc (desc_bytes >= qft_debug_pass_desc_size()), and
 * launch[0..5) = {threads, lds_bytes, grid, reads_workspace,
 * writes_workspace}.  Table pointers in the copy are NULL, except the
 * per-thread group-factor table pointer, which holds that table's byte
 * offset in the image qft_debug_tables returns (0: the pass has none).    */
int qft_debug_pass(int n, int cutoff, int norm, int layout, const qft_config_t *config,
                   int pass, void *out_desc, size_t desc_bytes, int *launch);

/* Copy the plan's twiddle-table image (in the plan's element type) into
 * out (out_bytes >= offsets[4]); offsets = {internal, low, high, end of the
 * high table, total} byte offsets (the per-thread group-factor tables follow
 * the high table).  Pass out = NULL to query offsets only.                  */
int qft_debug_tables(int n, int cutoff, int norm, int layout, const qft_config_t *config,
                     void *out, size_t out_bytes, size_t *offsets);

#ifdef __cplusplus
}
#endif
#endif /* QFT_MI355X_DEBUG_H */
