/*
 * fringe.h -- C ABI of the MI355X single-pulse fringe search (libfringe.so).
 *
 * The library searches complex visibilities for single pulses the way the
 * VOLKS2 pipeline does (paper, section "Fringe fitting" and section "Code
 * optimization", steps 5 and 6): for every baseline and every window of W
 * consecutive accumulation periods (APs), the visibilities x[t, f] of the
 * window (f = IF * n_chan + channel: all IFs form one band, one delay is
 * searched across them) are transformed to the delay / delay-rate grid
 *
 *   G[k_t, k_f] = sum_{u<W} sum_{f<F} x[t0+u, f]
 *                 * exp(-2 pi i (k_t u / M_t + k_f f / M_f)),
 *
 *   M_f = pad_freq * F   (the paper zero-pads its delay FFT 4x),
 *   M_t = pad_time * W   (rate axis; pad_time = 1 with k_t = 0 alone is the
 *                         paper's plain coherent sum over the window).
 *
 * The peak of P = |G|^2 (ties: lowest flat index k_t * M_f + k_f), the mean
 * power E = mean(P) (equal to sum |x|^2 by Parseval), amp = sqrt(P_peak) and
 * SNR = amp / sqrt(E) (0 when E = 0) are taken per window, and a window is a
 * candidate when SNR > snr_threshold (section "Detection rate": windows whose
 * normalised power exceeds a threshold).  Windows of length W start every
 * max(1, W/2) APs; a tail shorter than W is dropped.
 *
 * Every step of the search runs in HIP kernels on the GPU; there is no CPU
 * path.  The consumers of the candidate list (cross-window and
 * cross-baseline matching, localization) are host code, declared in
 * fringe_match.h.
 *
 * Conventions for every entry point:
 *   - returns 0 (FRINGE_OK) or a negative FRINGE_E_* code; never aborts or
 *     throws across the ABI; fringe_last_error() gives a detail message for
 *     the calling thread's last failure;
 *   - a plan is not thread-safe; separate plans may be used concurrently
 *     from separate threads on separate streams;
 *   - visibilities must be finite; NaN / Inf inputs give undefined results.
 */
#ifndef FRINGE_H
#define FRINGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------- */
#define FRINGE_OK             0
#define FRINGE_E_INVALID     -1  /* bad pointer, shape or parameter value          */
#define FRINGE_E_UNSUPPORTED -2  /* valid but not built: non power-of-two F or W,   */
                                 /* pad factors other than pad_freq 1/2/4,          */
                                 /* pad_time 1/2, M_f outside [64, 4096], W > 128   */
#define FRINGE_E_NOMEM       -3  /* the plan does not fit hbm_budget_bytes or HBM  */
#define FRINGE_E_HIP         -4  /* a HIP runtime call failed                       */
#define FRINGE_E_CAPACITY    -5  /* output capacity too small; *n_total is exact   */
#define FRINGE_E_STATE       -6  /* call out of order (e.g. results before search) */

/* ---- flags (fringe_params.flags) ----------------------------------------- */
#define FRINGE_STREAMING  0x1u   /* each fringe_search call is the next chunk      */
#define FRINGE_DUMP_GRID  0x2u   /* keep every window's full grid (tests; small)   */
#define FRINGE_PROFILE    0x4u   /* time every kernel launch with HIP events       */
#define FRINGE_PLAIN      0x8u   /* one window per launch (a baseline for timing;  */
                                 /* batch plans with windows of at most 64 APs)    */
#define FRINGE_GRAPH      0x10u  /* batch plans: capture a search's kernels in a  */
                                 /* HIP graph on a private stream, and replay it   */
                                 /* while the inputs (the d_vis pointers, so every */
                                 /* descriptor) are those of the captured search;  */
                                 /* new inputs are captured anew.  Not with        */
                                 /* STREAMING, PROFILE or PLAIN.                   */
#define FRINGE_DELAY_ONLY 0x20u  /* the paper's delay-only search (section "Code   */
                                 /* optimization", step 6): per window the APs'    */
                                 /* spectra summed coherently, the peak over the   */
                                 /* M_f delay bins of rate bin 0 and E = the mean  */
                                 /* power over those bins; k_rate = 0, rate_hz = 0 */
                                 /* and pad_time unused.  Windows of at most 64    */
                                 /* APs; not with DUMP_GRID.                       */
#define FRINGE_AUTOTUNE   0x40u  /* plans with windows of at most 64 APs: every    */
                                 /* class of scans (F, pads, longest window, on    */
                                 /* this device kind) takes its search mode and    */
                                 /* time chunk from the library's tune table; a    */
                                 /* class missing from it is tuned when the plan   */
                                 /* is made (each candidate timed on a synthetic   */
                                 /* sample of the class's shape, about a second    */
                                 /* per class; fringe_tune_load / _save keep the   */
                                 /* table across processes).  The chunk does not   */
                                 /* change results; the mode changes the delay     */
                                 /* transform's rounding only.                     */

/* One complex64 sample, identical in layout to torch.complex64 / numpy.complex64. */
typedef struct { float re, im; } fringe_cf32;

/* Opaque plan; owned by the library, released by fringe_plan_destroy. */
typedef struct fringe_plan_s* fringe_plan_t;

/* Shape of one scan (or, with FRINGE_STREAMING, of one chunk of a subarray's
 * stream).  Its visibility cube is complex64, C order
 * [n_baselines][n_ap][n_if][n_chan]; F = n_if * n_chan must be a power of
 * two.  ap_seconds (AP length) and chan_width_hz (channel width) only set the
 * physical units of the reported delay and rate. */
typedef struct {
  int32_t n_baselines, n_ap, n_if, n_chan;
  double ap_seconds, chan_width_hz;
} fringe_scan_desc;

/* Search parameters, shared by every scan of a plan. */
typedef struct {
  const int32_t* window_aps;   /* window lengths W in APs, strictly ascending powers of two, <= 128 */
  int32_t n_window_lengths;    /* 1..8                                                              */
  int32_t pad_freq;            /* M_f / F: 1, 2 or 4 (the paper uses 4)                             */
  int32_t pad_time;            /* M_t / W: 1 or 2                                                   */
  float snr_threshold;         /* candidate iff SNR > snr_threshold (strict), >= 0                  */
  uint64_t hbm_budget_bytes;   /* device bytes the plan may own; 0 = no limit beyond free HBM       */
  int64_t max_candidates;      /* device candidate buffer length (>= 0)                             */
  uint32_t flags;              /* FRINGE_* flags                                                    */
} fringe_params;

/* One window's result (a candidate, or any window via fringe_windows_get).
 * k_rate in [0, M_t), k_delay in [0, M_f); delay_s and rate_hz use signed
 * bins (bin >= M/2 means bin - M): delay_s = sk_delay / (M_f * chan_width_hz),
 * rate_hz = sk_rate / (M_t * ap_seconds).  energy is E (= sum |x|^2). */
typedef struct {
  int32_t scan, baseline, window_ap, t_start, k_rate, k_delay;
  float amp, snr, energy;
  int32_t reserved;
  double delay_s, rate_hz;
} fringe_candidate;

/* Sizes of a plan, from fringe_plan_check (no device work) or fringe_plan_info. */
typedef struct {
  int64_t n_windows;           /* windows of one full search (all scans, baselines, lengths) */
  int64_t device_bytes;        /* device memory the plan owns                                 */
  int64_t scratch_bytes;       /* of which transient work buffers                             */
  int32_t max_window_ap;       /* largest W                                                   */
  int32_t slab_baselines;      /* baselines processed per pass over the scratch               */
} fringe_plan_summary;

/* Validate scans and params and size the plan, without touching the GPU.
 * Returns FRINGE_OK and fills *out, or the error fringe_plan would return
 * for the same arguments (FRINGE_E_NOMEM only for an explicit budget). */
int fringe_plan_check(const fringe_scan_desc* scans, int32_t n_scans,
                      const fringe_params* params, fringe_plan_summary* out);

/* Build a plan on the current HIP device: validate, enumerate windows,
 * allocate all device memory within params->hbm_budget_bytes, upload the
 * twiddle tables.  scans[0..n_scans) and params (including window_aps) are
 * copied; the caller may free them afterwards.  *out receives the plan. */
int fringe_plan(const fringe_scan_desc* scans, int32_t n_scans,
                const fringe_params* params, fringe_plan_t* out);

/* Enqueue one search on hip_stream (a hipStream_t; NULL = default stream).
 * d_vis[s] is the device address of scan s's cube (layout above); the
 * caller owns it and keeps it valid and unchanged until the work on the
 * stream has completed.  With FRINGE_STREAMING, d_vis[s] is the next chunk
 * of subarray s (NULL: no chunk this call) and the windows reported are
 * those whose last AP lies in that chunk (D APs earlier with dedispersion
 * shifts up to D, fringe_set_shifts), windows spanning the previous chunk
 * included; start APs count from the first chunk.  The kernels read a chunk
 * where the caller holds it (with dedispersion shifts, from a copy); the
 * APs of it that the next call's windows reach back to are copied on the
 * stream during the call, so once the search has completed the chunk's
 * memory may be reused for the next one.  A search on another
 * stream than the plan's previous search first waits for that search.
 * Asynchronous: returns once the kernels are enqueued. */
int fringe_search(fringe_plan_t plan, const fringe_cf32* const* d_vis, void* hip_stream);

/* Wait for the plan's last search and copy its candidates, sorted by
 * (scan, baseline, window_ap, t_start), into host_out[0..capacity).
 * *n_total receives the number of candidates found.  If n_total exceeds
 * capacity or params->max_candidates, the first min(capacity,
 * max_candidates) in order are copied and FRINGE_E_CAPACITY is returned.
 * The search itself enqueues the copy of the count and of the first
 * min(max_candidates, 2048) records to pinned host memory, so up to that
 * many candidates come back with no further device transfer. */
int candidates_get(fringe_plan_t plan, fringe_candidate* host_out,
                   int64_t capacity, int64_t* n_total);

/* Results of chosen windows of the last search.  Window ids number the
 * windows in (scan, baseline, window length, start) order: id = scan_offset
 * + baseline * n_per_baseline + level_offset + j, j = t_start / stride.
 * (With FRINGE_STREAMING the ids number the windows of the last call.)
 * Waits for the search; copies n records into host_out. */
int fringe_windows_get(fringe_plan_t plan, const int64_t* window_ids, int64_t n,
                       fringe_candidate* host_out);

/* Window id <-> (scan, baseline, window_ap, t_start) for this plan. */
int fringe_window_id(fringe_plan_t plan, int32_t scan, int32_t baseline,
                     int32_t window_ap, int32_t t_start, int64_t* id);

/* Full grid G of one window (plans made with FRINGE_DUMP_GRID only):
 * M_t * M_f samples, row-major [k_t][k_f], into host_out[0..capacity). */
int fringe_grid_get(fringe_plan_t plan, int64_t window_id, fringe_cf32* host_out,
                    int64_t capacity);

/* Calibration and channel flags of scan s (a subarray, with FRINGE_STREAMING)
 * for the searches that follow (paper: Eq. (1), whose per-IF delay and phase
 * offsets are removed by multiplying each channel by
 * exp(-i (2 pi f dtau + dphi)); section "Code optimization", step 3).
 * d_gains: device address of n_baselines x F complex gains, [b][f] with
 * f = n * n_chan + c; every sample of baseline b, channel f is multiplied by
 * g[b][f] before the delay transform (0 flags a channel; a real factor
 * scales it).  E and SNR are those of the calibrated data.  The caller owns
 * the gains and keeps them valid and unchanged while searches that use them
 * may run; NULL returns to unit gains.  Errors: FRINGE_E_INVALID for a null
 * plan or a scan index out of range. */
int fringe_set_gains(fringe_plan_t plan, int32_t scan, const fringe_cf32* d_gains);

/* Dedispersion of scan s for the searches that follow (paper: section
 * "Code optimization", step 4: a time shift per frequency point for one DM
 * value).  d_shifts: device address of F int32 AP counts d_f >= 0; the
 * search sees x'[b][t][f] = x[b][t + d_f][f], and 0 where t + d_f runs past
 * the scan (values are clamped to [0, n_ap]).  Several DM trials of one cube
 * are several scans of one plan with the same visibility pointer and their
 * own shifts: one search call, one launch.  The caller owns the shifts and
 * keeps them valid and unchanged while searches that use them may run; NULL
 * removes them.  With FRINGE_STREAMING (shifts set before the plan's first
 * search; the library reads them once to size the subarray's stage for the
 * largest shift D, remaking the plan's buffers), a call reports the windows
 * whose last AP lies D APs before the end of the data received so far, so a
 * window is reported once its shifted reads have arrived: over the stream,
 * exactly the windows of a batch search of the concatenated APs that end
 * at least D APs before its end, with the same records.  Errors:
 * FRINGE_E_INVALID for a null plan or a scan out of range; FRINGE_E_STATE
 * for a streaming plan that has searched; FRINGE_E_UNSUPPORTED for
 * FRINGE_PLAIN plans, shifts above 2^20 APs and baselines (streaming: stages)
 * of 1 GiB or more of samples. */
int fringe_set_shifts(fringe_plan_t plan, int32_t scan, const int32_t* d_shifts);

/* Time chunk of scan's search (section "Parallelization": a scan is cut
 * into time ranges that are searched independently; here the ranges are
 * the work items of one search).  A work item searches the windows starting in its chunk
 * of APs and transforms W_max - 1 APs of halo besides, so longer chunks
 * transform fewer APs twice and shorter ones give more work items.  The
 * automatic choice (chunk 0, or the tune table's with FRINGE_AUTOTUNE)
 * fills the device with this plan's work alone; plans searched at the same
 * time on several streams (one per subarray in a server) share the device
 * and may do better with longer chunks.  Results are bit-identical for
 * every chunk.  chunk: 0, or a multiple of the search period (4 APs for
 * W_max <= 8, 16 up to 32, 32 for 64) in [64, 1024].  Before the plan's
 * first search (FRINGE_E_STATE after); the plan's device buffers are made
 * again.  FRINGE_E_UNSUPPORTED for plans with windows longer than 64 APs,
 * whose chunk is fixed.  fringe_plan_get_chunk reads the chunk in use. */
int fringe_plan_set_chunk(fringe_plan_t plan, int32_t scan, int32_t chunk);
int fringe_plan_get_chunk(fringe_plan_t plan, int32_t scan, int32_t* chunk);

/* Dedispersion as a pass of its own, for plans without shifts (paper:
 * section "Code optimization", step 4): d_out[b][t][f] = d_in[b][t + d_f][f],
 * 0 where t + d_f >= n_ap, d_f = d_shifts[f] clamped to [0, n_ap] (the
 * semantics of fringe_set_shifts).  d_in and d_out: device cubes of
 * n_baselines x n_ap x n_freq complex64 in the layout above (n_freq = F =
 * n_if * n_chan), not overlapping; d_shifts: device array of n_freq int32.
 * The caller owns all three and keeps them valid until the work on
 * hip_stream (a hipStream_t; NULL = default stream) has completed.
 * Asynchronous.  Searching the result without shifts gives exactly what
 * fringe_set_shifts gives on the original; the pass reads each input line
 * once per output row, where the in-kernel shifts read it once per delay-bin
 * class of the search, so it is the faster route for the delay-only search,
 * whose kernel is bound by those reads, at the price of a cube-sized buffer.
 * Errors: FRINGE_E_INVALID for null pointers, sizes below 1 or overlapping
 * buffers; FRINGE_E_HIP for a failed launch. */
int fringe_dedisperse(const fringe_cf32* d_in, fringe_cf32* d_out, int32_t n_baselines,
                      int32_t n_ap, int32_t n_freq, const int32_t* d_shifts, void* hip_stream);

/* Kernel times of the last search of a plan made with FRINGE_PROFILE,
 * measured with HIP events recorded on the search's stream around each
 * launch (waits for the search).  Times in milliseconds, summed over the
 * launches of each kernel; the counts are the launches. */
typedef struct {
  double delay_ms, rate_ms, finalize_ms, compact_ms;
  int32_t delay_launches, rate_launches, finalize_launches, compact_launches;
} fringe_profile;

int fringe_profile_get(fringe_plan_t plan, fringe_profile* out);

/* Sizes of an existing plan. */
int fringe_plan_info(fringe_plan_t plan, fringe_plan_summary* out);

/* One entry of the tune table (FRINGE_AUTOTUNE): a class of scans and the
 * launch configuration chosen for it on this kind of device. */
typedef struct {
  int32_t n_freq, pad_freq;    /* F = n_if * n_chan, M_f / F                     */
  int32_t pad_time;            /* M_t / W; 0 for the delay-only search           */
  int32_t log2_wmax;           /* longest window, at most 64 APs                 */
  int32_t spectra;             /* 1: the delay spectra go through HBM and the    */
                               /* rate kernels read them; 0: one fused kernel    */
                               /* transforms and searches                        */
  int32_t chunk;               /* APs per work item (plans on grids too small to */
                               /* fill the device with it take less)             */
  float ms_fused, ms_spectra;  /* the tuning sample's best time in each mode      */
                               /* (ms; < 0: not a candidate)                      */
} fringe_tune_entry;

/* Merge the tune table stored in the JSON file at path (written by
 * fringe_tune_save) into the library's; entries for other device kinds are
 * kept but unused here.  Errors: FRINGE_E_INVALID for an unreadable or
 * malformed file (the table is then unchanged). */
int fringe_tune_load(const char* path);

/* Write the library's tune table (every entry, every device kind) as JSON.
 * Errors: FRINGE_E_INVALID when the file cannot be written. */
int fringe_tune_save(const char* path);

/* Empty the library's tune table. */
void fringe_tune_clear(void);

/* The tune entries a plan made with FRINGE_AUTOTUNE uses, one per class of
 * its scans, into out[0..capacity); *n receives their number
 * (FRINGE_E_CAPACITY if it exceeds capacity).  0 entries for other plans. */
int fringe_plan_tuning(fringe_plan_t plan, fringe_tune_entry* out, int32_t capacity, int32_t* n);

/* Release every resource of the plan (waits for its outstanding work).
 * NULL is ignored. */
void fringe_plan_destroy(fringe_plan_t plan);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * search of fringe_plan + fringe_search + candidates_get for ONE scan, same
 * kernels and same results, with no plan and no allocation of any kind:
 * every work buffer lives in a static device array of the library
 * (64 MiB per GPU, held by each GPU the library runs on until the process
 * ends).  scan and params as for fringe_plan (params->window_aps up to 64
 * APs; hbm_budget_bytes and max_candidates ignored; flags 0 or
 * FRINGE_DELAY_ONLY).  d_vis: the scan's device cube (layout above);
 * d_out: device array of capacity records that receives the first
 * min(capacity, total) candidates in key order; d_total: device int64 that
 * receives the total count.  The caller owns all three and keeps them valid
 * until the work on hip_stream (a hipStream_t; NULL = default stream) has
 * completed.  Asynchronous.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race, so
 * the caller orders them.  Errors: FRINGE_E_INVALID for null pointers, a
 * negative capacity or other flags; the errors of fringe_plan for the
 * shape; FRINGE_E_NOMEM when the scan's work buffers (about 8 B per window
 * and 64-bin delay class, 16 B per window, 4 B per AP and baseline) exceed
 * the 64 MiB; FRINGE_E_HIP for a failed launch. */
int fringe_search_noalloc(const fringe_scan_desc* scan, const fringe_params* params,
                          const fringe_cf32* d_vis, fringe_candidate* d_out, int64_t capacity,
                          int64_t* d_total, void* hip_stream);

/* Static description of an error code. */
const char* fringe_strerror(int code);

/* Detail message of the calling thread's last failed call ("" if none). */
const char* fringe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FRINGE_H */
