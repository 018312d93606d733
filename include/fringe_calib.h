/*
 * fringe_calib.h -- calibration helpers of libfringe that prepare the
 * per-baseline, per-channel gains fringe_set_gains (fringe.h) folds into
 * the search.
 */
#ifndef FRINGE_CALIB_H
#define FRINGE_CALIB_H

#include <stdint.h>

#include "fringe.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Auto-spectrum amplitude normalisation (paper, section "Fringe fitting":
 * the amplitude of each frequency point divided by the auto-spectrum
 * dispersions of the two stations, the Mk4 / HOPS convention):
 *
 *   d_gains_out[b][f] = g_in[b][f] * (abar_i^2[f] * abar_j^2[f])^(-1/4),
 *   abar_s^2[f] = (1 / n_spectra) * sum_k d_auto[s][k][f]^2,
 *
 * for baseline b with stations (i, j) = (d_pairs[2b], d_pairs[2b + 1]);
 * g_in = d_gains_in[b][f], or 1 when d_gains_in is NULL (it may equal
 * d_gains_out: the normalisation is then applied in place).  A zero product
 * (a station without power in the channel), or a station index outside
 * [0, n_stations), gives a zero gain: the channel is flagged on that
 * baseline.  Pass the result to fringe_set_gains.
 *   d_auto:   device, n_stations x n_spectra x n_freq float32 auto-spectra
 *             (real), channel fastest, f = IF * n_chan + channel;
 *   d_pairs:  device, n_baselines x 2 int32 station indices;
 *   d_gains_in / d_gains_out: device, n_baselines x n_freq complex64.
 * The caller owns every buffer and keeps them valid until the work on
 * hip_stream (a hipStream_t; NULL = default stream) has completed.
 * Asynchronous.  Errors: FRINGE_E_INVALID for null pointers, sizes below 1
 * or gain arrays that overlap without being the same; FRINGE_E_HIP for a
 * failed launch. */
int fringe_autospectrum_gains(const float* d_auto, int32_t n_stations, int32_t n_spectra,
                              int32_t n_freq, const int32_t* d_pairs, int32_t n_baselines,
                              const fringe_cf32* d_gains_in, fringe_cf32* d_gains_out,
                              void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FRINGE_CALIB_H */
