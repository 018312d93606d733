/*
 * fringe_match.h -- C ABI of the single-pulse consumers of libfringe.so:
 * matching of candidate windows into single pulses, and their localization
 * from delays.  Host code (these calls run on the calling CPU thread and
 * touch no device memory); they take the candidate list that
 * candidates_get returns.
 *
 * Matching (paper, section "Detection rate": the criteria a single pulse
 * must meet).  The criteria name no grouping rule;
 * groups here are anchored at their strongest member (so that a long-lived
 * RFI signal, whose windows overlap one another for seconds, cannot chain
 * distinct pulses into one):
 *   1. Baseline pulses.  Among the candidates of one (scan, baseline),
 *      repeatedly take the strongest remaining window (highest SNR; ties:
 *      the shorter window, then the earlier start) and every remaining
 *      window whose AP span [t_start, t_start + window_ap) shares an AP with
 *      it.  The group is a pulse of that baseline when its windows have at
 *      least min_windows distinct lengths (the paper: present in at least 2
 *      of its window series).  Its span [t_lo, t_hi) is the union of the
 *      windows' spans; its representative is the anchor window.
 *   2. Single pulses.  Among the baseline pulses of one scan, repeatedly take
 *      the strongest remaining one (by its representative window, ties: the
 *      lower baseline) and every remaining one whose span shares an AP with
 *      the anchor's span.  The group is a single pulse when it holds at
 *      least min_baselines distinct baselines (the paper: 5).  A baseline
 *      with several pulses in the group is represented by its strongest.
 *
 * Localization (paper, section "Localization", Eq. (2)): least squares for
 * the offsets (dra, ddec) from the a priori position in
 *   tau_b - tau_cal_b = (dtau/dra)_b dra + (dtau/ddec)_b ddec
 * over a pulse's baselines b, and the same solve leaving out each baseline
 * in turn (section "Localization accuracy": the check for a baseline whose
 * delay is wrong, since the solutions that include it deviate; the fit
 * without it has the smallest residual).
 *
 * Conventions as in fringe.h: 0 or a negative FRINGE_E_* code, detail in
 * fringe_last_error(); every call is reentrant (no shared state).
 */
#ifndef FRINGE_MATCH_H
#define FRINGE_MATCH_H

#include <stdint.h>

#include "fringe.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Matching criteria. */
typedef struct {
  int32_t min_windows;    /* distinct window lengths per baseline pulse, >= 1 (paper: 2) */
  int32_t min_baselines;  /* distinct baselines per single pulse, >= 1 (paper: 5)         */
} fringe_match_params;

/* One baseline of one single pulse.  The window fields (window_ap ..
 * rate_hz) are those of the baseline's representative candidate; t_lo,
 * t_hi, n_windows and n_lengths describe the baseline pulse it represents
 * (its span, its candidate count and distinct lengths).  pulse numbers the
 * single pulses from 0 in (scan, first AP of the group, order found) order. */
typedef struct {
  int32_t scan, pulse, baseline, window_ap, t_start, k_rate, k_delay;
  int32_t t_lo, t_hi, n_windows, n_lengths;
  float amp, snr;
  int32_t reserved;
  double delay_s, rate_hz;
} fringe_pulse;

/* Match candidates[0..n) (any order; window_ap >= 1, t_start >= 0) into
 * single pulses.  Writes the rows, in (pulse, baseline) order, to
 * out[0..capacity); *n_rows and *n_pulses receive the exact counts.  If
 * n_rows exceeds capacity, the first capacity rows are written and
 * FRINGE_E_CAPACITY is returned.  out may be NULL when capacity is 0 (a
 * sizing call).  Errors: FRINGE_E_INVALID for null pointers, n < 0,
 * criteria below 1, or a candidate with window_ap < 1, t_start < 0, a span
 * reaching past INT32_MAX or a non-finite SNR. */
int fringe_match(const fringe_candidate* candidates, int64_t n,
                 const fringe_match_params* params, fringe_pulse* out, int64_t capacity,
                 int64_t* n_rows, int64_t* n_pulses);

/* Least squares of Eq. (2) over n >= 2 baselines.  tau[i]: the residual
 * delay minus the fine-calibration delay (s); dtau_dra[i], dtau_ddec[i]:
 * the partials at the a priori position (s/rad).  sol[0..2) receives
 * (dra, ddec) in rad and *rms the RMS of the n delay residuals.  If
 * loo != NULL (2 n doubles) and loo_rms != NULL (n doubles) and n >= 3,
 * loo[2 i .. 2 i + 2) and loo_rms[i] receive the solution and the RMS over
 * the n - 1 kept baselines with baseline i left out (NaN where those
 * baselines do not fix both offsets); with n = 2 they are not written.
 * Errors: FRINGE_E_INVALID for null pointers, n < 2, non-finite input, or
 * partials that do not fix both offsets (collinear columns). */
int fringe_localize(const double* tau, const double* dtau_dra, const double* dtau_ddec,
                    int32_t n, double* sol, double* rms, double* loo, double* loo_rms);

/* Partials of the geometric delay tau_g = t_2 - t_1 = -(b . s) / c for n
 * baselines b_xyz[3 i .. 3 i + 3) = r_2 - r_1 (Earth-fixed metres, c =
 * 299792458 m/s) toward a source at (ra, dec) whose Greenwich hour angle
 * is gast - ra (radians), with s = (cos dec cos h, -cos dec sin h, sin dec),
 * h = gast - ra.  The a priori geometry of a small offset solve: no
 * precession, nutation, polar motion or aberration.  Where the correlator's
 * delay has the opposite sign (t_1 - t_2), negate both partials.
 * Errors: FRINGE_E_INVALID for null pointers or n < 0. */
int fringe_delay_partials(const double* b_xyz, int32_t n, double gast, double ra, double dec,
                          double* dtau_dra, double* dtau_ddec);

#ifdef __cplusplus
}
#endif

#endif /* FRINGE_MATCH_H */
