/* Continuous-batching search of streamed subarrays (C ABI).
 *
 * The paper's pipeline overlaps the loading of one time range with the
 * search of others (section "Parallelization": idle calculation processes
 * take the next time range while others load theirs).  Here a correlator
 * delivers each subarray's visibilities as a stream of fixed-length chunks
 * already in device memory, and the server searches them as they come: one
 * streaming plan (fringe.h, FRINGE_STREAMING) and one HIP stream of default
 * priority per subarray, and a worker thread of its own that admits
 * waiting chunks (first come, first served across subarrays; a subarray's
 * chunks in order, one in flight at a time, since its plan holds the halo of
 * the last chunk), launches their searches, and collects the candidates of
 * finished ones.  The caller submits chunks and polls results from any
 * thread; timestamps are CLOCK_MONOTONIC nanoseconds (the clock of
 * fringe_monotonic_ns), so arrival-to-result latency can be measured
 * against the caller's own clock.
 */
#ifndef FRINGE_SERVE_H
#define FRINGE_SERVE_H

#include <stdint.h>

#include "fringe.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fringe_server_s* fringe_server_t;

/* One finished chunk. */
typedef struct {
  int32_t sub;            /* subarray                                           */
  int32_t status;         /* FRINGE_OK, or the error of its search / copy-out    */
  int64_t tag;            /* the caller's tag from fringe_server_submit          */
  int64_t n_candidates;   /* candidates returned with it (<= n_total)            */
  int64_t n_total;        /* candidates found (more than max_candidates: cut)    */
  int64_t n_windows;      /* windows the search reported                         */
  int64_t t_submit_ns;    /* fringe_server_submit accepted it                    */
  int64_t t_launch_ns;    /* its search was enqueued                             */
  int64_t t_done_ns;      /* the worker saw the search finish, candidates copied */
} fringe_serve_result;

/* Monotonic clock (CLOCK_MONOTONIC) in nanoseconds. */
int64_t fringe_monotonic_ns(void);

/* Create a server on the current HIP device for n_subs subarrays whose
 * chunks have the shapes subs[0..n_subs) (n_ap = APs per chunk).  params as
 * for fringe_plan; FRINGE_STREAMING is implied, FRINGE_PLAIN and
 * FRINGE_GRAPH are refused (FRINGE_E_UNSUPPORTED), FRINGE_DELAY_ONLY,
 * FRINGE_AUTOTUNE and FRINGE_PROFILE are passed on.  time_chunk: APs per
 * work item of every plan's search (fringe_plan_set_chunk; 0 = each plan's
 * automatic choice).  max_inflight: chunks searched at once over all
 * subarrays (1..n_subs; 0 = n_subs).  The worker thread starts at once.
 * Errors: FRINGE_E_INVALID (arguments), those of fringe_plan and
 * fringe_plan_set_chunk, FRINGE_E_HIP. */
int fringe_server_create(const fringe_scan_desc* subs, int32_t n_subs,
                         const fringe_params* params, int32_t time_chunk,
                         int32_t max_inflight, fringe_server_t* out);

/* Dedispersion shifts of subarray sub (fringe_set_shifts on its plan: F
 * int32 APs on the device, read once; windows are then reported once the
 * data D = max shift APs past their end have arrived).  Only before the
 * first fringe_server_submit (FRINGE_E_STATE after). */
int fringe_server_set_shifts(fringe_server_t server, int32_t sub, const int32_t* d_shifts);

/* Queue the next chunk of subarray sub: d_chunk is its device cube
 * [n_baselines][n_ap][n_if][n_chan] complex64, which the caller keeps valid
 * and unchanged until the chunk's result has been returned by
 * fringe_server_poll (the search reads it on the subarray's stream; work
 * the caller enqueued to produce it must have completed).  tag is returned
 * with the result.  Never blocks on the device; thread-safe. */
int fringe_server_submit(fringe_server_t server, int32_t sub, int64_t tag,
                         const fringe_cf32* d_chunk);

/* Take finished chunks, oldest first: up to capacity results into out, and
 * the candidates of those results, concatenated in the same order, into
 * cands[0..cand_capacity) (sorted per chunk as by candidates_get).  A result
 * is returned only with all its copied candidates; *n_out results and
 * *n_cands candidates are written.  FRINGE_E_CAPACITY when the oldest
 * result alone needs more than cand_capacity (then *n_cands holds that
 * need and nothing is taken).  Non-blocking; thread-safe. */
int fringe_server_poll(fringe_server_t server, fringe_serve_result* out, int32_t capacity,
                       int32_t* n_out, fringe_candidate* cands, int64_t cand_capacity,
                       int64_t* n_cands);

/* Chunks submitted and not yet taken by fringe_server_poll (waiting,
 * searching, or finished and held). */
int fringe_server_pending(fringe_server_t server, int64_t* n);

/* Stop the worker (after the searches in flight complete), release the
 * plans, streams and results.  Results not yet polled are dropped. */
int fringe_server_destroy(fringe_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* FRINGE_SERVE_H */
