/*
 * qft_metrics.h - accuracy of the approximate QFT, on the device and in
 * closed form (libqft.so).
 *
 * The range-k AQFT (Sec. 2, "Approximate QFT") trades accuracy for
 * controlled-phase gates.  Sec. 4 judges it by the relative L2 error, the
 * fidelity and the leakage out of the dominant bin.  This header gives:
 *  - qft_compare: those metrics between a transform's output and a
 *    reference output already in device memory (for instance the exact
 *    transform of the same input), in one reading pass over both arrays;
 *  - qft_execute_compare: a transform whose last pass also takes those
 *    metrics against a reference, so that its output is not read back;
 *  - qft_aqft_expected_error: the expected relative L2 error of the range-k
 *    AQFT against the exact transform for inputs with i.i.d. complex
 *    Gaussian amplitudes, in closed form (host only);
 *  - qft_select_cutoff: the smallest cutoff whose expected error meets a
 *    budget (host only), so that callers can pick k by accuracy.
 */
#ifndef QFT_MI355X_METRICS_H
#define QFT_MI355X_METRICS_H

#include <stddef.h>

#include "qft.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Slots of the metrics array qft_compare writes (doubles).                  */
#define QFT_METRIC_REL_L2 0    /* ||y - ref||_2 / ||ref||_2 (0 if both zero)    */
#define QFT_METRIC_MAX_ERR 1   /* max_k |y_k - ref_k| / RMS(ref)                */
#define QFT_METRIC_FIDELITY 2  /* |<ref, y>|^2 / (||ref||^2 ||y||^2) (Sec. 4)   */
#define QFT_METRIC_LEAKAGE 3   /* 1 - |y_k*|^2 / ||y||^2, k* = argmax |ref_k|,
                                  lowest index on ties (Sec. 4)                  */
#define QFT_METRIC_NORM_Y 4    /* ||y||_2                                       */
#define QFT_METRIC_NORM_REF 5  /* ||ref||_2                                     */
#define QFT_METRIC_ARGMAX 6    /* k* as a double                                */
#define QFT_METRIC_COUNT 7

/* Device workspace qft_compare needs for 2^n elements, in bytes.           */
size_t qft_compare_workspace_bytes(int n);

/* Compare y with ref (device arrays of 2^n elements of the element type in
 * `layout`, QFT_C64 or QFT_C128; other layout bits are ignored) and write
 * QFT_METRIC_COUNT doubles to metrics_dev (device memory, 8-byte aligned),
 * asynchronously on `stream`.  All sums are formed in FP64: fixed-size
 * per-workgroup partials, combined in a fixed order, so a call is
 * deterministic.  workspace: device memory of qft_compare_workspace_bytes(n)
 * bytes, 8-byte aligned, caller-owned; calls that share it must be ordered
 * on one stream.  Returns QFT_OK, QFT_ERR_INVALID (n out of range) or
 * QFT_ERR_POINTER (NULL or misaligned pointer).                           */
int qft_compare(const void *y, const void *ref, int n, int layout, void *workspace,
                double *metrics_dev, qft_stream_t stream);

/* Device workspace qft_execute_compare needs for this plan, in bytes (0 for
 * a NULL plan).                                                            */
size_t qft_execute_compare_workspace_bytes(const qft_plan_t *plan);

/* Transform dev_ptr in place as qft_execute_ws does (workspace NULL = the
 * plan's own), and write to metrics_dev the QFT_METRIC_COUNT metrics of
 * qft_compare between the output y and `ref` (2^n elements of the plan's
 * element type, in the plan's output order, for instance the exact
 * transform of the same input), asynchronously on `stream`.  Sec. 4's
 * accuracy measures of the range-k AQFT taken as the transform runs: with
 * the fused schedule the last pass compares the tiles it stores with ref
 * (it reads ref once and never reads y back), and a short reduction of its
 * per-wave FP64 partials follows; with the gate schedule a separate
 * comparison pass follows the transform.  The partials are combined in a
 * fixed order, so a call is deterministic; the sums are the same as
 * qft_compare's up to FP64 rounding order (the maxima and the argmax are
 * identical).  ref must not overlap dev_ptr or the workspace
 * (QFT_ERR_INVALID).
 * cmp_workspace: device memory of qft_execute_compare_workspace_bytes(plan)
 * bytes, 8-byte aligned, caller-owned; calls that share it must be ordered
 * on one stream.  Errors as qft_execute_ws, and QFT_ERR_POINTER for a NULL
 * or misaligned ref, cmp_workspace or metrics_dev.                          */
int qft_execute_compare(qft_plan_t *plan, void *dev_ptr, void *workspace, const void *ref,
                        void *cmp_workspace, double *metrics_dev, qft_stream_t stream);

/* Expected relative L2 error E||(U - U_k) x|| / E||U x|| of the range-k
 * AQFT U_k against the exact QFT U (both unitary) for inputs with i.i.d.
 * complex Gaussian amplitudes: sqrt(||U - U_k||_F^2 / N), evaluated in
 * closed form from the phases the dropped gates would add (cost 2^M * M
 * terms with M = n - 1 - k, under a second at M = 20).  0 for the exact
 * transform; a negative value when M exceeds 20 (such cutoffs err by more
 * than 10 % at any n) or n is out of range.                                 */
double qft_aqft_expected_error(int n, int cutoff);

/* Smallest cutoff k in [0, n-1] whose expected error is <= budget (fewest
 * controlled-phase gates at that accuracy).  The expected error falls as k
 * grows, so the search walks k down from n - 1 and stops at the first
 * failure, or at M = n - 1 - k = 20 (see above).  Returns -1 for an invalid
 * n or a negative budget.                                                  */
int qft_select_cutoff(int n, double rel_l2_budget);

#ifdef __cplusplus
}
#endif
#endif /* QFT_MI355X_METRICS_H */
