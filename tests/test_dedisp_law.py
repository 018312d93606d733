"""The dispersion law behind dedisp.dm_shifts, pinned from first principles.

A radio wave of frequency f crossing a cold plasma of electron density n_e
travels at the group velocity v_g = c sqrt(1 - f_p^2 / f^2), with the plasma
frequency f_p^2 = n_e e^2 / (4 pi^2 eps0 m_e).  Over a path of L parsecs at
n_e = 1 cm^-3 (a dispersion measure of L pc cm^-3) its travel time is
L / v_g, and the pulse at f arrives (L / c) (1 / sqrt(1 - f_p^2 / f^2) - 1)
after an infinitely high frequency.  The test computes these delays from
the CODATA constants (no dispersion constant in it), exactly in double
precision (expm1 / log1p), and checks the shifts dm_shifts gives in APs:
each is the nearest integer to the physical delay difference to the band's
highest channel.  A planted mistake in the law (a 1/f instead of 1/f^2,
the lowest channel as the reference, a frequency in Hz where MHz is meant,
a rounding down) fails."""

import numpy as np
import pytest

from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts

# CODATA 2018 (exact where the SI fixes them) and the IAU parsec
E_CHARGE = 1.602176634e-19        # C
M_ELECTRON = 9.1093837015e-31     # kg
EPS0 = 8.8541878128e-12           # F / m
C_LIGHT = 299792458.0             # m / s
PARSEC = 3.0856775814913673e16    # m


def physical_delay_s(freq_hz, dm):
    """Arrival delay (s) at freq_hz after an infinite frequency, through
    dm pc of plasma at 1 electron per cm^3, from the group velocity."""
    n_e = 1e6                                             # m^-3
    fp2 = n_e * E_CHARGE ** 2 / (4 * np.pi ** 2 * EPS0 * M_ELECTRON)
    x = fp2 / np.asarray(freq_hz, dtype=np.float64) ** 2
    return dm * PARSEC / C_LIGHT * np.expm1(-0.5 * np.log1p(-x))


def check_law(shift_fn):
    cases = [(1.6e9, 8, 32, 0.5e6, 1.024e-3, 100.0),
             (1.6e9, 8, 32, 0.5e6, 1.024e-3, 500.0),
             (0.3e9, 4, 64, 0.25e6, 0.512e-3, 57.0),
             (4.9e9, 16, 16, 1e6, 1e-3, 1000.0)]
    for f0, n_if, n_chan, bw, ap, dm in cases:
        f = channel_freqs_hz(f0, n_if, n_chan, bw)
        want = (physical_delay_s(f, dm) - physical_delay_s(f.max(), dm)) / ap
        got = shift_fn(dm, f, ap)
        assert got.shape == f.shape
        # nearest AP, away from rounding ties (the physics and the usual
        # dispersion constant agree to a few parts per million)
        clear = np.abs(want - np.floor(want) - 0.5) > 1e-3 + 1e-5 * np.abs(want)
        assert clear.mean() > 0.9
        np.testing.assert_array_equal(got[clear], np.rint(want[clear]).astype(np.int64))
        assert np.all(np.abs(got - want) <= 0.5 + 1e-3 + 1e-5 * np.abs(want))
        assert got[np.argmax(f)] == 0 and want.max() > 10


def test_dm_shifts_follow_the_group_delay():
    check_law(dm_shifts)


@pytest.mark.parametrize("mistake", ["inverse_f", "lowest_reference", "hz_units", "floor"])
def test_planted_law_mistakes_fail(mistake):
    k = 4.148808e3

    def bad(dm, freqs_hz, ap_seconds):
        f = np.asarray(freqs_hz, dtype=np.float64) / 1e6
        if mistake == "inverse_f":
            dt = k * dm * (f ** -1 - f.max() ** -1) / 1e3
        elif mistake == "lowest_reference":
            dt = k * dm * (f ** -2 - f.min() ** -2)
        elif mistake == "hz_units":
            dt = k * dm * ((f * 1e6) ** -2 - (f.max() * 1e6) ** -2)
        else:
            dt = k * dm * (f ** -2 - f.max() ** -2)
            return np.maximum(np.floor(dt / ap_seconds), 0).astype(np.int32)
        return np.maximum(np.rint(dt / ap_seconds), 0).astype(np.int32)

    with pytest.raises(AssertionError):
        check_law(bad)
