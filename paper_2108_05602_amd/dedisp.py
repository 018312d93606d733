"""Dedispersion shifts for fringe_set_shifts.

The cold-plasma dispersion delay of frequency f relative to f_ref is
    dt = K_DM * DM * (f^-2 - f_ref^-2),   K_DM = 4.148808e3 s MHz^2 pc^-1 cm^3,
(f in MHz, DM in pc cm^-3).  A channel's shift is that delay in APs,
rounded to the nearest AP, with the highest frequency as the reference so
every shift is >= 0 (the paper's step 4: one time shift per frequency point
for a given DM value).  Host-side helper: the shifts are uploaded by the
caller and applied inside the search kernels.
"""

from __future__ import annotations

import numpy as np

K_DM_S_MHZ2 = 4.148808e3


def channel_freqs_hz(f0_hz: float, n_if: int, n_chan: int, chan_width_hz: float,
                     if_width_hz: float | None = None) -> np.ndarray:
    """Frequencies of the concatenated channels f = n * n_chan + c: IF n starts
    at f0 + n * if_width (contiguous IFs by default), channel c at + c * width."""
    if_width_hz = n_chan * chan_width_hz if if_width_hz is None else if_width_hz
    n = np.arange(n_if)[:, None]
    c = np.arange(n_chan)[None, :]
    return (f0_hz + n * if_width_hz + c * chan_width_hz).reshape(-1)


def dm_shifts(dm: float, freqs_hz, ap_seconds: float, f_ref_hz: float | None = None) -> np.ndarray:
    """Per-channel AP shifts (int32, >= 0) of dispersion measure dm."""
    f = np.asarray(freqs_hz, dtype=np.float64) / 1e6
    f_ref = (np.max(f) if f_ref_hz is None else f_ref_hz / 1e6)
    dt = K_DM_S_MHZ2 * float(dm) * (f ** -2 - f_ref ** -2)
    return np.maximum(np.rint(dt / ap_seconds), 0).astype(np.int32)
