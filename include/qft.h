/*
 * qft.h - C ABI of the MI355X (gfx950) QFT->FFT library (libqft.so).
 *
 * The library computes the discrete Fourier transform of a 2^n-element
 * complex array by executing the gate schedule of the n-qubit quantum Fourier
 * transform circuit (Hadamard butterflies, controlled-phase diagonals, final
 * qubit-reversal swaps) on the array as a state vector, optionally truncated
 * to the range-k approximate QFT.  The paper this follows is "Not Your Usual
 * FFT: QFT->FFT via Classical Quantum-Circuit Simulation" (Markidis et al.).
 *
 * Conventions (paper Sec. 2 and Sec. 3):
 *  - element i of the array is the amplitude of basis state |b_{n-1}...b_0>
 *    with qubit q_j = bit j of i (Sec. 3 step 1; Sec. 2 one-wire gate on q_j
 *    = I_{2^{n-1-j}} (x) U (x) I_{2^j});
 *  - forward sign: y_k = s * sum_j x_j exp(-2 pi i j k / N) (Sec. 2,
 *    w_N = exp(-2 pi i / N), R_k = diag(1, exp(-2 pi i / 2^k)));
 *  - the scale s is chosen by `norm` (Sec. 3 steps 3 and 4);
 *  - the cutoff keeps controlled phases whose control-target distance is
 *    <= cutoff (Sec. 2 "Approximate QFT"); the paper's scale_in
 *    normalisation (Sec. 3 step 1) is not applied: the map is linear, so the
 *    result equals the paper's decoded output up to rounding.
 *
 * Memory: all data pointers are device pointers (hipMalloc'd or torch CUDA
 * tensors) owned by the caller unless stated.  Arrays are interleaved
 * (re, im) complex, contiguous, 2^n elements, complex64 (2 x float) or
 * complex128 (2 x double), at least 16-byte aligned.  Transforms are in place.
 *
 * Streams: `qft_stream_t` is a hipStream_t passed as void* (NULL = the null
 * stream).  Execute calls only enqueue work; they never synchronise the host.
 *
 * Errors: functions return QFT_OK (0) or a negative QFT_ERR_* code, or NULL
 * for constructors; qft_last_error() returns the calling thread's last
 * message.  No C++ exception crosses this interface.
 */
#ifndef QFT_MI355X_H
#define QFT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qft_plan_s qft_plan_t;
typedef void *qft_stream_t; /* hipStream_t */

/* ---- norm: output scale (Sec. 3 steps 3-4) ------------------------------ */
#define QFT_NORM_UNITARY 0 /* y = DFT_N x / sqrt(N)  (the unit-norm QFT U)   */
#define QFT_NORM_NONE 1    /* y = DFT_N x            (unnormalised FFT)      */
#define QFT_NORM_INV_N 2   /* y = DFT_N x / N        (1/N convention)        */

/* ---- layout flags (OR them together) ------------------------------------ */
#define QFT_C64 0x0            /* complex64 data, FP32 arithmetic             */
#define QFT_C128 0x1           /* complex128 data, FP64 arithmetic            */
#define QFT_ORDER_NATURAL 0x0  /* y[k] = bin k: final swaps applied (Fig. 1)  */
#define QFT_ORDER_BITREV 0x2   /* y[rev_n(k)] = bin k: swaps left to the
                                  caller as an index permutation (Sec. 3
                                  step 2)                                     */
#define QFT_SCHEDULE_FUSED 0x0 /* fused HBM passes (default)                  */
#define QFT_SCHEDULE_GATES 0x4 /* one sweep per gate: H, controlled-R_m and
                                  SWAP in circuit order (Fig. 1), unfused     */
#define QFT_PLAN_NO_WORKSPACE 0x8 /* the plan allocates no workspace: run it
                                  with qft_execute_ws (qft_execute then fails
                                  with QFT_ERR_POINTER if one is needed)      */
#define QFT_PLAN_TUNED 0x20    /* build the plan with the tuning table's
                                  entry for its shape when there is one
                                  (qft_tune.h); without this flag, and
                                  always with an explicit configuration, the
                                  table is not consulted, so a plan does not
                                  depend on what was tuned before          */
#define QFT_INVERSE 0x10       /* the inverse transform: the same circuit with
                                  every controlled phase conjugated, R_m ->
                                  R_m^*, i.e. y_k = s * sum_j x_j
                                  exp(+2 pi i j k / N) when exact.  H and the
                                  swaps are real and the (A)QFT matrix is
                                  symmetric, so this is its adjoint: with
                                  QFT_NORM_UNITARY it undoes the forward plan
                                  of the same cutoff; QFT_NORM_INV_N gives
                                  the usual 1/N inverse FFT scale            */

#define QFT_CUTOFF_EXACT (-1) /* any cutoff < 0 or >= n-1 is exact            */
#define QFT_MAX_QUBITS 31
#define QFT_MAX_PASSES 8

/* ---- error codes --------------------------------------------------------- */
#define QFT_OK 0
#define QFT_ERR_INVALID (-1)     /* bad argument value                        */
#define QFT_ERR_UNSUPPORTED (-2) /* valid but unsupported combination         */
#define QFT_ERR_NOMEM (-3)       /* device allocation failed                  */
#define QFT_ERR_HIP (-4)         /* HIP runtime or launch error               */
#define QFT_ERR_POINTER (-5)     /* NULL or misaligned pointer                */
#define QFT_ERR_BUSY (-6)        /* resource limit (admission, queue)         */

/* Kernel configuration of the fused schedule.  Zero fields mean "default";
 * a negative spec_log2 / rev_spec_log2 requests 0 spectator bits.
 * tile_log2:   elements per workgroup tile (2^tile_log2), 1..15
 * radix_log2:  qubits applied in registers between LDS exchanges, 1..5
 * spec_log2:   contiguous low-order elements kept in each tile of the
 *              high-order passes (coalescing width 2^spec_log2)
 * rev_spec_log2: contiguous output elements per run in the final
 *              bit-reversing pass (natural order only)
 * nontemporal: streaming (non-temporal) loads and stores, which do not
 *              keep the data in the caches: 0 = planner's choice (on passes
 *              whose tiles read whole 128-byte lines, when the state is
 *              at least 256 MiB and so does not stay in the 256 MB
 *              Infinity Cache between passes), 1 = never, 2 = on every pass
 *              whose tiles read whole 128-byte lines
 * pass_bits:   qubits of each HBM pass, most significant pass first,
 *              summing to n (all zero = planner's choice: the fewest passes,
 *              middle passes as wide as the tile allows, the rest split
 *              between the first and the last pass, whose rows lie furthest
 *              apart in memory)
 * pass_tile_log2: tile bits of each pass, most significant pass first (0 =
 *              planner's choice: tile_log2, or tile_log2 + 1 for the passes
 *              below which other qubits lie, in complex64 plans of at least
 *              2^26 elements, so that their rows hold 2^(tile - bits)
 *              contiguous elements; such 512-thread workgroups run the
 *              four-wave form of the kernels, two per CU).  A pass's
 *              spectator bits are its tile bits minus its qubits.          */
typedef struct qft_config {
  int tile_log2;
  int radix_log2;
  int spec_log2;
  int rev_spec_log2;
  int nontemporal;
  int pass_bits[QFT_MAX_PASSES];
  int pass_tile_log2[QFT_MAX_PASSES];
} qft_config_t;

/* Description of a plan.  Gate counts are those of the circuit before any
 * fusion (the paper's aggregate 1- and 2-qubit counters, Sec. 3.1).          */
typedef struct qft_plan_info {
  int n;
  int cutoff;          /* effective cutoff: n-1 for the exact transform      */
  int norm;
  int layout;
  int num_passes;      /* kernel launches per execute (fused) or gate sweeps */
  int pass_lo[QFT_MAX_PASSES];   /* lowest qubit applied by pass p           */
  int pass_bits[QFT_MAX_PASSES]; /* qubits applied by pass p                 */
  int pass_spec[QFT_MAX_PASSES]; /* spectator (coalescing) bits of pass p    */
  int pass_reverse[QFT_MAX_PASSES]; /* pass p writes bit-reversed addresses  */
  int pass_kernel[QFT_MAX_PASSES];  /* 0: the generic pass kernel; 1..10:
                                       the compile-time two-group kernel,
                                       1 + 5 * (below-pass diagonal) +
                                       (stages of the last group - 1);
                                       11..16: the compile-time three-group
                                       kernel, 11 + 3 * (below-pass
                                       diagonal) + (qubits - 11);
                                       17..21: the two-group kernel with a
                                       store exchange (the last pass of a
                                       bit-reversed-order plan), 16 + (stages
                                       of the last group)                    */
  int pass_streaming[QFT_MAX_PASSES]; /* pass p uses non-temporal access    */
  qft_config_t config;
  long long gates_h, gates_cr, gates_swap;
  size_t state_bytes;     /* 2^n * element size                              */
  size_t workspace_bytes; /* plan-owned scratch (natural order, >1 pass)     */
  size_t table_bytes;     /* plan-owned twiddle tables on the device         */
  size_t hbm_bytes;       /* algorithmic HBM bytes per execute: 2 * state
                             bytes per pass (read + write)                   */
} qft_plan_info_t;

/* ---- core ---------------------------------------------------------------- */

/* Build a plan for 2^n-point transforms (host planning in FP64, then a
 * one-time upload of its twiddle tables to the current device).
 * n: 1..QFT_MAX_QUBITS.  cutoff: AQFT range k (see QFT_CUTOFF_EXACT).
 * norm: QFT_NORM_*.  layout: dtype | order | schedule flags.
 * Returns NULL on error (see qft_last_error).                               */
qft_plan_t *qft_plan(int n, int cutoff, int norm, int layout);

/* As qft_plan with an explicit kernel configuration (NULL = default).      */
qft_plan_t *qft_plan_config(int n, int cutoff, int norm, int layout,
                            const qft_config_t *config);

/* Transform dev_ptr (2^n elements, in place) asynchronously on `stream`.
 * Uses the plan's own workspace, so executes of one plan must be ordered on
 * one stream.                                                              */
int qft_execute(qft_plan_t *plan, void *dev_ptr, qft_stream_t stream);

/* As qft_execute with a caller-owned workspace of info.workspace_bytes
 * (may be NULL when that is 0), so one plan can run on several streams.    */
int qft_execute_ws(qft_plan_t *plan, void *dev_ptr, void *workspace,
                   qft_stream_t stream);

/* As qft_execute_ws (workspace NULL = the plan's own), and also write the
 * input's L2 norm ||x||_2 as one double to norm_dev (device memory, 8-byte
 * aligned) on the same stream.  This is the paper's scale_in (Sec. 3 step
 * 1): the transform is linear, so encoding x / scale_in, evolving and
 * decoding by scale_in gives the same output up to rounding, and the norm is
 * returned as metadata.  The fused schedule sums |x|^2 in its first pass
 * (no extra pass over the state); the gate schedule adds one reading sweep.
 * The first call allocates a small plan-owned buffer of partial sums (8
 * bytes per 64 threads of the first pass); calls of one plan must be
 * ordered on one stream.  Errors as qft_execute_ws, and QFT_ERR_POINTER for
 * a NULL or misaligned norm_dev.                                           */
int qft_execute_norm(qft_plan_t *plan, void *dev_ptr, void *workspace,
                     double *norm_dev, qft_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * qft_execute_norm, but the partial sums live in a static device array of
 * QFT_NORM_SCRATCH_DOUBLES doubles (8 MiB, one per GPU, held until the
 * process ends) instead of a plan-owned buffer, so this call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine; it records
 * no per-launch timing events).  The plan (tables, workspace) is built
 * beforehand as usual.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU race and must be ordered by the
 * caller (one stream, or events).  Every partial is rewritten before it is
 * read, so no clearing is needed.  Returns QFT_ERR_UNSUPPORTED when the plan
 * needs more partial sums than the array holds (not the case for any
 * default plan up to n = 31), else as qft_execute_norm.                   */
#define QFT_NORM_SCRATCH_DOUBLES (1u << 20)
int qft_execute_norm_static(qft_plan_t *plan, void *dev_ptr, void *workspace,
                            double *norm_dev, qft_stream_t stream);

/* Free the plan and its device memory (NULL-safe).  The caller must ensure
 * no enqueued execute of the plan is still pending.                         */
void qft_destroy(qft_plan_t *plan);

/* Thread-local message describing the last error ("" if none).             */
const char *qft_last_error(void);

int qft_plan_info(const qft_plan_t *plan, qft_plan_info_t *out);

/* Device memory the plan holds, in bytes: its twiddle tables, its workspace
 * (none for QFT_PLAN_NO_WORKSPACE plans) and, once qft_execute_norm has run,
 * its norm partial sums.  The state array is the caller's and is not
 * counted.  For admission by HBM budget (the plan / execute split of
 * Sec. 3.1).  0 for NULL.                                                   */
size_t qft_plan_device_bytes(const qft_plan_t *plan);

/* Run only the host planner (no device use) and describe the plan that
 * qft_plan_config would build.                                             */
int qft_plan_describe(int n, int cutoff, int norm, int layout,
                      const qft_config_t *config, qft_plan_info_t *out);

/* ---- measurement --------------------------------------------------------- */

/* When enabled, qft_execute records HIP events around every kernel launch
 * it enqueues (one more event per launch, plus one per execute).  The events
 * of all executes since the last qft_plan_pass_times call are kept, and
 * reused after it: call it now and then while timing is on.  Executes of a
 * timed plan must be ordered on one stream.                                 */
int qft_plan_set_timing(qft_plan_t *plan, int enable);
/* Synchronises on the recorded events and returns the mean milliseconds per
 * execute of each pass in ms[0..count) (count = min(max, num_passes)) and
 * the number of timed executes; the accumulators are then cleared.          */
int qft_plan_pass_times(qft_plan_t *plan, double *ms, int max, long long *execs);

/* ---- batched uneven sizes (one graph launch) ----------------------------- */

/* Transform count arrays, dev_ptrs[i] with plans[i], with one graph launch.
 * The tiles of all transforms are grouped by pass level, then by register
 * radix, workgroup size and kernel shape; each group is one kernel launch
 * over the tiles of many transforms (one tile per workgroup), and the
 * launches run level by level, so a transform's pass p+1 starts after every
 * pass-p tile is done and no workgroup waits on another.  A transform's
 * passes take the last levels (with the largest plan having maxP passes, a
 * plan of P passes runs pass p at level maxP - P + p): one-pass transforms
 * run beside the last passes of the large ones.  The first call for a given
 * (plans, dev_ptrs) set builds the work list (and allocates one workspace per
 * natural-order multi-pass transform) and captures the launches into a HIP
 * graph; later calls replay the graph.  Plans must be fused-schedule plans
 * of one element type.  Results equal those of each plan's own qft_execute
 * bit for bit.  Destroying a plan drops the cached sets that use it.  At
 * most 64 sets stay cached: a new set beyond that synchronises the device
 * once and releases the oldest.  The graph's launches of one pass level are
 * spread, largest first, over the caller's stream and three streams of the
 * set, joined before the next level.                                        */
int qft_execute_batch(qft_plan_t *const *plans, void *const *dev_ptrs,
                      int count, qft_stream_t stream);

#define QFT_BATCH_EAGER 0x1 /* enqueue the launches directly, no graph         */
int qft_execute_batch_ex(qft_plan_t *const *plans, void *const *dev_ptrs,
                         int count, int flags, qft_stream_t stream);

/* ---- device input generation (Philox-4x32-10, Salmon et al. 2011) -------- */
#define QFT_RNG_GAUSSIAN 0 /* re, im ~ N(0, 1) (Box-Muller in FP64)          */
#define QFT_RNG_UNIFORM 1  /* re, im ~ U[-1, 1)                              */
/* Fill dev_ptr (2^n elements, layout dtype bit) with amplitude i drawn from
 * Philox(counter = (i, stream_id), key = seed).                              */
int qft_fill_random(void *dev_ptr, int n, int layout, int dist, uint64_t seed,
                    uint64_t stream_id, qft_stream_t stream);

/* ---- lengths that are not powers of two (Sec. 3 step 1) ----------------- */
/* The method maps N amplitudes onto n = ceil(log2 N) qubits and allocates
 * 2^n of them; the transform is then DFT_{2^n} of the input padded with
 * zeros, not DFT_N.  qft_pad copies `count` elements from src to dst and
 * zero-fills dst[count, 2^n), in one pass, asynchronously on `stream`.
 * src and dst are device arrays of the layout's element type (QFT_C64 or
 * QFT_C128); they must not overlap.  count <= 2^n.  Returns QFT_OK,
 * QFT_ERR_INVALID or QFT_ERR_POINTER.                                       */
int qft_pad(const void *src, size_t count, void *dst, int n, int layout, qft_stream_t stream);

/* Smallest n with 2^n >= count (count >= 1), or -1.                         */
int qft_qubits_for(size_t count);

#ifdef __cplusplus
}
#endif
#endif /* QFT_MI355X_H */
