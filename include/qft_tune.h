/*
 * qft_tune.h - autotuner and tuning cache of libqft.so.
 *
 * The tuner times candidate kernel configurations (qft_config_t: tile size,
 * register radix = number of qubits fused per register group, spectator
 * widths) on the device and keeps the fastest per plan shape in an
 * in-memory table.  A plan uses the table entry for its shape only when it
 * is built with the QFT_PLAN_TUNED layout flag and no explicit
 * configuration; otherwise plans do not depend on the table.  The table can
 * be saved to and loaded from a text file of JSON lines; lines that do not
 * parse, or that name another GPU architecture, are skipped.  The radix
 * stops at 32 (five fused qubits): a 64-element register block would hold
 * 128 complex64 data registers per lane.
 */
#ifndef QFT_MI355X_TUNE_H
#define QFT_MI355X_TUNE_H

#include <stddef.h>

#include "qft.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Time every candidate configuration of the built-in grid (tile_log2 8..14,
 * radix_log2 3..5, spectator widths 2..5; combinations the planner rejects
 * are skipped) for the plan shape (n, cutoff, norm, layout) on `data`
 * (2^n elements of the layout's element type; its contents are
 * overwritten), `reps` timed executes each after one warm-up.  The fastest
 * is stored in the tuning table and returned.                               */
int qft_tune(int n, int cutoff, int norm, int layout, void *data, int reps,
             qft_config_t *best, double *best_ms);

/* Tune one configuration shared by all transforms of a batch: for each
 * candidate of the batch grid (tile_log2 8..14, radix_log2 3..5, spectator
 * widths 2..4), plans (n[i], cutoff[i], norm, layout) are built with it and
 * the batch on data[i] is timed through qft_execute_batch (graph launch,
 * after one call that captures it).  The winner and its time are returned;
 * the per-shape table is not changed.                                       */
int qft_tune_batch(const int *n, const int *cutoff, int count, int norm, int layout,
                   void *const *data, int reps, qft_config_t *best, double *best_ms);

/* Look up / insert entries by hand (no device use).                        */
int qft_tune_lookup(int n, int cutoff, int layout, qft_config_t *out);
int qft_tune_insert(int n, int cutoff, int layout, const qft_config_t *config, double ms);
int qft_tune_clear(void);

/* Persist the table (JSON lines) / merge a saved table.  load returns the
 * number of entries read (>= 0) or an error code.                            */
int qft_tune_save(const char *path);
int qft_tune_load(const char *path);

#ifdef __cplusplus
}
#endif
#endif /* QFT_MI355X_TUNE_H */
