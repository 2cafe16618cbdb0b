/*
 * qft_serve.h - continuous-batching request server of libqft.so.
 *
 * A server replays a stream of transform requests in real time.  Requests
 * are released at their arrival times into a FIFO queue and admitted, in
 * order, as soon as an in-flight slot is free and the HBM budget fits: the
 * budget is charged once with the device memory of the server's resident
 * plans (their twiddle tables) and then with the state buffer plus
 * workspace of every request in flight.  Admitted requests are enqueued
 * on a pool of HIP streams, so that requests arriving while others run are
 * overlapped on the device.  Each request generates its input on the device
 * (Philox-4x32-10, see qft_fill_random), runs its cached plan and records a
 * completion event; completion frees its budget and slot.  Latency is
 * arrival -> completion detected by the host.
 *
 * Plans are built ahead of the run (qft_server_prepare), so plan
 * construction stays outside the measured latencies, as the paper excludes
 * plan construction from its timings (Sec. 4 experimental setup).
 */
#ifndef QFT_MI355X_SERVE_H
#define QFT_MI355X_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "qft.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qft_server_s qft_server_t;

typedef struct qft_request {
  int n;            /* qubits (2^n amplitudes)                               */
  int cutoff;       /* AQFT range, or QFT_CUTOFF_EXACT                       */
  int norm;         /* QFT_NORM_*                                            */
  int layout;       /* dtype | order | QFT_INVERSE flags (fused schedule) */
  int dist;         /* input distribution, QFT_RNG_*                         */
  uint64_t seed;    /* Philox key of the request's input                     */
  double arrival;   /* seconds after the start of the run                    */
  void *out;        /* optional device buffer (2^n elements) that receives a
                       copy of the result; NULL = result discarded           */
} qft_request_t;

typedef struct qft_request_result {
  double arrival;   /* seconds after the start of the run                    */
  double admitted;  /* when its work was enqueued                            */
  double completed; /* when the host saw its completion event                */
  int status;       /* QFT_OK or an error code                               */
  int stream;       /* index of the stream it ran on                         */
  size_t bytes;     /* HBM bytes reserved for it (state + workspace)         */
} qft_request_result_t;

typedef struct qft_server_stats {
  long long completed;
  long long failed;
  size_t peak_reserved_bytes;
  int peak_inflight;
  double wall_seconds;
  double hbm_bytes;  /* algorithmic HBM bytes of all transforms + inputs     */
  size_t plan_bytes; /* device memory of the resident plans, charged against
                        the budget for the whole run (peak_reserved_bytes
                        includes it)                                         */
} qft_server_stats_t;

/* hbm_budget_bytes: admission budget; max_inflight: in-flight slots;
 * num_streams: HIP streams of the pool (>= 1).  The device is the current
 * one.  Returns NULL on error.                                              */
qft_server_t *qft_server_create(size_t hbm_budget_bytes, int max_inflight, int num_streams);
void qft_server_destroy(qft_server_t *server);

/* Build and cache the plans the requests need (outside any timing).        */
int qft_server_prepare(qft_server_t *server, const qft_request_t *reqs, int count);

/* Replay `count` requests (sorted by arrival) in real time and block until
 * all have completed.  results[i] describes reqs[i].  Fails with
 * QFT_ERR_NOMEM when the resident plans alone exceed the budget.            */
int qft_server_run(qft_server_t *server, const qft_request_t *reqs, int count,
                   qft_request_result_t *results, qft_server_stats_t *stats);

/* The same scheduler driven by a simulated device and a virtual clock (no
 * GPU use): request i needs bytes[i] of budget and runs for service[i]
 * seconds once admitted.  For testing admission and ordering logic.         */
int qft_server_simulate(size_t hbm_budget_bytes, int max_inflight, const double *arrival,
                        const size_t *bytes, const double *service, int count,
                        qft_request_result_t *results, qft_server_stats_t *stats);

#ifdef __cplusplus
}
#endif
#endif /* QFT_MI355X_SERVE_H */
