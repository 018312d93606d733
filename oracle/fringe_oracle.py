"""Reference implementation of the single-pulse fringe search, in complex128.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It is deliberately slow and plain: every transform
is the direct DFT written as a dense matrix product, every peak is found by a
brute-force argmax, so that a reader can check it against the paper by eye.

What is computed (paper: section "Fringe fitting", the search function G with
its phase model Eq. (1); section "Code optimization", steps 5 and 6; section
"Detection rate", the threshold on each window series):

  For one baseline with visibilities x[t, f] (t = accumulation period, f the
  concatenated IF x channel index, all IFs treated as one band), a window of
  W consecutive APs starting at t0 gives the delay / delay-rate grid

      G[k_t, k_f] = sum_{u<W} sum_{f<F} x[t0+u, f]
                    * exp(-2 pi i (k_t u / M_t + k_f f / M_f)),

  with M_f = pad_freq * F delay bins and M_t = pad_time * W rate bins (the
  zero padding of the paper's delay FFT, and of the rate transform the
  delay-rate search adds).  P = |G|^2; the peak is the argmax of P, ties broken
  by the lowest flat index k_t * M_f + k_f; E = mean(P); amp = sqrt(P_peak);
  SNR = amp / sqrt(E) (0 when E = 0).  A window is a candidate when SNR
  exceeds the threshold.  Windows of length W start every max(1, W // 2) APs;
  a tail shorter than W is dropped.

The delay-only search (the paper's own scheme, without a rate axis) takes
the same steps on the single row k_t = 0: the window's APs summed
coherently, one zero-padded delay transform, the peak over the delay axis,
E = the mean power over that axis (delay_only_row).

Readings of points the paper leaves open: all channels are summed, IF
calibration terms are zero, the rate axis has its own zero padding, windows
overlap by half, SNR is the peak amplitude over the root of the mean grid
power, ties go to the lowest flat index, an all-zero window has peak (0, 0)
and SNR 0.  Each function below names the passage it follows.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "window_stride",
    "window_starts",
    "delay_dft_matrix",
    "rate_dft_matrix",
    "delay_spectra",
    "window_grid",
    "grid_peak",
    "signed_bin",
    "WindowResult",
    "search_window",
    "delay_only_row",
    "search_window_delay_only",
    "search_baseline",
    "search_scan",
    "calibrate",
    "autospectrum_gains",
    "dedisperse",
    "TABLE_DTYPE",
]


def window_stride(window_ap: int) -> int:
    """Start-to-start distance of windows of one length: half the length
    (50 % overlap), and 1 for single-AP windows.

    Paper: section "Fringe fitting" builds time segments of several window
    sizes by summing APs; the stride is not stated there, so the half-window
    overlap of the benchmark configurations is used.
    """
    return max(1, window_ap // 2)


def window_starts(n_ap: int, window_ap: int) -> np.ndarray:
    """All start APs t0 = j * stride with t0 + W <= n_ap, ascending."""
    s = window_stride(window_ap)
    if n_ap < window_ap:
        return np.zeros(0, dtype=np.int64)
    return np.arange(0, n_ap - window_ap + 1, s, dtype=np.int64)


def delay_dft_matrix(n_freq: int, m_f: int) -> np.ndarray:
    """A_f[f, k] = exp(-2 pi i k f / M_f) for f < F, k < M_f.

    Paper: section "Fringe fitting", the search function G sums
    S(n, j) exp(-i Phi) with Phi = 2 pi (f0_n + f_j - f_ref) dtau (Eq. 1,
    calibration terms zero); evaluating Phi on the delay grid
    dtau = k / (M_f * df) of an FFT zero-padded by M_f / F gives this matrix
    (up to the constant phase of f0 - f_ref, which leaves |G| unchanged).
    """
    f = np.arange(n_freq, dtype=np.float64)[:, None]
    k = np.arange(m_f, dtype=np.float64)[None, :]
    return np.exp(-2j * np.pi * (f * k) / m_f)


def rate_dft_matrix(window_ap: int, m_t: int) -> np.ndarray:
    """A_t[k, u] = exp(-2 pi i k u / M_t) for k < M_t, u < W.

    The delay-rate axis: the transform over the window's APs, zero-padded
    to M_t = pad_time * W.  Its row k = 0 is the plain coherent sum of the
    window's APs, which is the paper's own combination (section "Code
    optimization", step 6).
    """
    k = np.arange(m_t, dtype=np.float64)[:, None]
    u = np.arange(window_ap, dtype=np.float64)[None, :]
    return np.exp(-2j * np.pi * (k * u) / m_t)


def delay_spectra(x_b: np.ndarray, pad_freq: int) -> np.ndarray:
    """Y[t, k_f] = sum_f x[t, f] exp(-2 pi i k_f f / M_f), every AP.

    Paper: section "Code optimization", step 5 (a transform along frequency
    for each AP, zero-padded by the padding factor of section "Fringe
    fitting").  x_b has shape (T, F); the result is complex128 (T, M_f).
    """
    x_b = np.asarray(x_b, dtype=np.complex128)
    n_freq = x_b.shape[1]
    return x_b @ delay_dft_matrix(n_freq, pad_freq * n_freq)


def window_grid(y: np.ndarray, t0: int, window_ap: int, pad_time: int) -> np.ndarray:
    """G[k_t, k_f] for the window [t0, t0 + W) from the delay spectra Y.

    The time sum of step 6 (section "Code optimization"), generalised from
    the rate-0 sum to all M_t rate bins.  Shape (M_t, M_f), complex128.
    """
    seg = y[t0:t0 + window_ap]
    if seg.shape[0] != window_ap:
        raise ValueError("window runs past the end of the data")
    return rate_dft_matrix(window_ap, pad_time * window_ap) @ seg


@dataclass
class WindowResult:
    k_rate: int
    k_delay: int
    amp: float
    snr: float
    energy: float
    peak_power: float
    margin: float  # (P1 - P2) / P1 over distinct bins, 1.0 if undefined


def grid_peak(g: np.ndarray, duplicate_rate_rows: bool = False) -> WindowResult:
    """Peak of |G|^2 with lowest-flat-index tie-break, mean power, SNR.

    Paper: section "Code optimization", step 6 (maximum amplitude over the
    delay axis, here over the delay-rate grid) and section "Detection rate"
    (a normalised power compared with a threshold; its normalisation is not
    given, and the grid's own mean power is used).

    `duplicate_rate_rows` marks grids whose rows are identical by
    construction (a one-AP window padded to two rate bins); the margin to
    the runner-up is then taken over the first row only, since the second
    row repeats it exactly in any arithmetic.
    """
    p = (g.real * g.real) + (g.imag * g.imag)
    m_f = p.shape[1]
    flat = int(np.argmax(p))  # first occurrence == lowest flat index
    k_t, k_f = divmod(flat, m_f)
    p1 = float(p.flat[flat])
    e = float(p.mean())
    amp = math.sqrt(p1)
    snr = amp / math.sqrt(e) if e > 0.0 else 0.0
    if e == 0.0:
        # all-zero window: peak at (0, 0), amplitude 0, never a candidate
        k_t, k_f, amp, snr = 0, 0, 0.0, 0.0
    q = p[:1] if duplicate_rate_rows else p
    if q.size > 1 and p1 > 0.0:
        second = np.partition(q.ravel(), -2)[-2]
        margin = (p1 - float(second)) / p1
    else:
        margin = 1.0
    return WindowResult(k_t, k_f, amp, snr, e, p1, margin)


def signed_bin(k: int, m: int) -> int:
    """FFT-frequency convention: bins at or above M/2 are negative."""
    return k - m if k >= m // 2 else k


def search_window(x_b: np.ndarray, t0: int, window_ap: int,
                  pad_freq: int, pad_time: int) -> WindowResult:
    """One window straight from the raw visibilities (both DFTs direct)."""
    seg = np.asarray(x_b[t0:t0 + window_ap], dtype=np.complex128)
    y = delay_spectra(seg, pad_freq)
    g = window_grid(y, 0, window_ap, pad_time)
    return grid_peak(g, duplicate_rate_rows=(window_ap == 1 and pad_time > 1))


def delay_only_row(x_seg: np.ndarray, pad_freq: int, a_f=None) -> np.ndarray:
    """The paper's own search function of one window, without a rate axis:

        G_0[k_f] = sum_{f<F} (sum_{u<W} x[u, f]) exp(-2 pi i k_f f / M_f),

    the window's APs summed coherently and transformed along frequency with
    the zero padding of the delay transform.  Paper: section "Code
    optimization", step 6 (the APs of a window summed, then the maximum
    amplitude along the delay axis) with step 5 and the padding of section
    "Fringe fitting".  x_seg has shape (W, F); the result has shape (1, M_f)
    so that grid_peak applies unchanged (its mean power is then the mean
    over the delay axis, = sum_f |sum_u x[u, f]|^2 by Parseval).  a_f, if
    given, is delay_dft_matrix(F, M_f), built once by the caller.
    """
    x_seg = np.asarray(x_seg, dtype=np.complex128)
    n_freq = x_seg.shape[1]
    if a_f is None:
        a_f = delay_dft_matrix(n_freq, pad_freq * n_freq)
    s = x_seg.sum(axis=0)
    return (s @ a_f)[None, :]


def search_window_delay_only(x_b: np.ndarray, t0: int, window_ap: int,
                             pad_freq: int, a_f=None) -> WindowResult:
    """One window of the delay-only search (rate bin 0 only)."""
    seg = np.asarray(x_b[t0:t0 + window_ap])
    if seg.shape[0] != window_ap:
        raise ValueError("window runs past the end of the data")
    return grid_peak(delay_only_row(seg, pad_freq, a_f))


TABLE_DTYPE = np.dtype([
    ("scan", np.int32), ("baseline", np.int32), ("window_ap", np.int32),
    ("t_start", np.int32), ("k_rate", np.int32), ("k_delay", np.int32),
    ("amp", np.float64), ("snr", np.float64), ("energy", np.float64),
    ("delay_s", np.float64), ("rate_hz", np.float64),
    ("margin", np.float64),
])


def search_baseline(x_b: np.ndarray, window_aps, pad_freq: int, pad_time: int,
                    ap_seconds: float, chan_width_hz: float,
                    scan: int = 0, baseline: int = 0,
                    delay_only: bool = False) -> np.ndarray:
    """Every window of one baseline, in (window length, start) order.

    The delay transform is done once per AP and shared by all windows
    (section "Code optimization": step 5 once, step 6 per window size).
    With delay_only, every window is searched by delay_only_row (rate bin 0,
    pad_time unused).
    """
    x_b = np.asarray(x_b)
    n_ap, n_freq = x_b.shape
    m_f = pad_freq * n_freq
    rows = []
    if delay_only:
        a_f = delay_dft_matrix(n_freq, m_f)
        for w in sorted(int(v) for v in window_aps):
            for t0 in window_starts(n_ap, w):
                r = search_window_delay_only(x_b, int(t0), w, pad_freq, a_f)
                rows.append((scan, baseline, w, int(t0), r.k_rate, r.k_delay,
                             r.amp, r.snr, r.energy,
                             signed_bin(r.k_delay, m_f) / (m_f * chan_width_hz), 0.0,
                             r.margin))
        return np.array(rows, dtype=TABLE_DTYPE)
    y = delay_spectra(x_b, pad_freq)
    for w in sorted(int(v) for v in window_aps):
        m_t = pad_time * w
        a_t = rate_dft_matrix(w, m_t)
        for t0 in window_starts(n_ap, w):
            g = a_t @ y[t0:t0 + w]
            r = grid_peak(g, duplicate_rate_rows=(w == 1 and pad_time > 1))
            rows.append((scan, baseline, w, int(t0), r.k_rate, r.k_delay,
                         r.amp, r.snr, r.energy,
                         signed_bin(r.k_delay, m_f) / (m_f * chan_width_hz),
                         signed_bin(r.k_rate, m_t) / (m_t * ap_seconds),
                         r.margin))
    return np.array(rows, dtype=TABLE_DTYPE)


def calibrate(vis: np.ndarray, gains) -> np.ndarray:
    """x'[b, t, f] = g[b, f] x[b, t, f]: per-baseline, per-channel complex gains
    applied to every AP before the search.  Paper: Eq. (1) and section
    "Fringe fitting" (the per-IF instrumental delay and phase offsets enter the
    phase model; removing them multiplies each channel by
    exp(-i (2 pi f dtau + dphi))), section "Code optimization" step 3 (the
    calibration applied ahead of the search); a gain of 0 flags a channel.
    vis has shape (B, T, F), gains (B, F)."""
    vis = np.asarray(vis, dtype=np.complex128)
    g = np.asarray(gains, dtype=np.complex128)
    if g.shape != (vis.shape[0], vis.shape[2]):
        raise ValueError("gains must have shape (baselines, channels)")
    return vis * g[:, None, :]


def autospectrum_gains(auto, pairs) -> np.ndarray:
    """Per baseline (i, j) and frequency point f, the amplitude normalisation
    by the two stations' auto-spectrum dispersions,

        g[b, f] = (abar_i^2[f] * abar_j^2[f]) ** (-1/4),

    abar_i^2[f] being the mean over station i's auto-spectra a_i[k, f] of
    their squares (0 where either station's is 0: the channel is flagged).
    Paper: section "Fringe fitting" (each frequency point's amplitude
    normalised, as in the Mk4 format of HOPS, by the auto-spectrum
    dispersion of the two stations).  auto has shape (n_stations,
    n_spectra, F), real; pairs gives (i, j) per baseline.  The result, shape
    (B, F), serves as the gains of calibrate / search_scan."""
    a = np.asarray(auto, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("auto must have shape (stations, spectra, channels)")
    disp = np.mean(a * a, axis=1)                    # abar^2, (n_stations, F)
    out = np.zeros((len(pairs), a.shape[2]))
    for b, (i, j) in enumerate(pairs):
        prod = disp[i] * disp[j]
        pos = prod > 0.0
        out[b, pos] = prod[pos] ** -0.25
    return out


def dedisperse(vis: np.ndarray, shifts) -> np.ndarray:
    """x'[b, t, f] = x[b, t + d_f, f], and 0 where t + d_f runs past the data:
    each channel moved earlier by its dispersion delay d_f >= 0 (in APs)
    relative to the reference (highest) frequency.  Paper: section "Code
    optimization", step 4 (dedispersion of the buffer for one DM value: a
    time shift per frequency point).  vis has shape (B, T, F), shifts (F,)."""
    vis = np.asarray(vis, dtype=np.complex128)
    d = np.asarray(shifts, dtype=np.int64)
    b_count, n_ap, n_freq = vis.shape
    if d.shape != (n_freq,) or np.any(d < 0):
        raise ValueError("shifts must be F non-negative AP counts")
    out = np.zeros_like(vis)
    for f in range(n_freq):
        k = int(d[f])
        if k < n_ap:
            out[:, :n_ap - k, f] = vis[:, k:, f]
    return out


def search_scan(vis: np.ndarray, window_aps, pad_freq: int, pad_time: int,
                snr_threshold: float, ap_seconds: float, chan_width_hz: float,
                scan: int = 0, baselines=None, delay_only: bool = False, gains=None,
                shifts=None):
    """Full search of one scan.

    vis has shape (B, T, n_if, n_chan) (or (B, T, F)); the frequency index
    is f = n * n_chan + c, so all IFs form one band (section "Fringe
    fitting": one delay across all IFs).  With gains (shape (B, F)), the
    visibilities are calibrated first (calibrate), with shifts (shape (F,))
    dedispersed (dedisperse; the two commute).  Returns (table, candidates): the
    per-window table in key order (baseline, window length, start) and the
    windows whose SNR exceeds the threshold (strictly), same order.
    """
    vis = np.asarray(vis)
    b_count, n_ap = vis.shape[0], vis.shape[1]
    flat = vis.reshape(b_count, n_ap, -1)
    if gains is not None:
        flat = calibrate(flat, gains)
    if shifts is not None:
        flat = dedisperse(flat, shifts)
    if baselines is None:
        baselines = range(b_count)
    tables = [search_baseline(flat[b], window_aps, pad_freq, pad_time,
                              ap_seconds, chan_width_hz, scan=scan, baseline=b,
                              delay_only=delay_only)
              for b in baselines]
    table = np.concatenate(tables) if tables else np.zeros(0, TABLE_DTYPE)
    cands = table[table["snr"] > snr_threshold]
    return table, cands
