"""Pins of the CPU reference against facts fixed by the paper and by the
mathematics of the DFT, not against itself.

Each check is a plain function of the reference module so that the
planted-mistake tests at the bottom can run the same checks against a
deliberately broken copy and confirm that some check catches it.
"""

import json
import math
import os
import types

import numpy as np
import pytest
from scipy import special, stats

import oracle.fringe_oracle as fo
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_x(rng, w, f):
    return rng.standard_normal((w, f)) + 1j * rng.standard_normal((w, f))


def _grid(mod, x, pad_f, pad_t):
    w = x.shape[0]
    y = mod.delay_spectra(x, pad_f)
    return mod.window_grid(y, 0, w, pad_t)


# ---------------------------------------------------------------- checks ---

def check_c1_closed_form(mod):
    """Noise-free C1: exact peak bins, amplitudes, SNRs, candidate list."""
    gold = json.load(open(os.path.join(GOLDEN, "c1_noise_free.json")))
    spec = synth.c1(noise=False)
    v = spec.full()
    table, cands = mod.search_scan(v, [gold["window_ap"]], gold["pad_freq"],
                                   gold["pad_time"], gold["snr_threshold"],
                                   spec.ap_seconds, spec.chan_width_hz)
    assert len(table) == gold["n_windows"]
    assert list(table["t_start"]) == list(range(0, 61, gold["stride"]))
    assert [int(c) for c in cands["t_start"]] == [c["t_start"] for c in gold["candidates"]]
    for row, g in zip(cands, gold["candidates"]):
        assert (int(row["k_rate"]), int(row["k_delay"])) == (g["k_rate"], g["k_delay"])
        assert row["amp"] == pytest.approx(g["amp"], rel=1e-6)
        assert row["snr"] == pytest.approx(g["snr"], rel=1e-6)
        assert row["energy"] == pytest.approx(g["energy"], rel=1e-6)
    rest = table[~np.isin(table["t_start"], cands["t_start"])]
    o = gold["other_windows"]
    assert np.all(rest["k_rate"] == o["k_rate"]) and np.all(rest["k_delay"] == o["k_delay"])
    assert np.all(rest["amp"] == 0.0) and np.all(rest["snr"] == 0.0)


def check_library_fft(mod):
    """G equals numpy's 2-D FFT of the zero-padded window (P3) and row 0
    equals the FFT of the coherent AP sum, the paper's own scheme (P4)."""
    rng = np.random.default_rng(7)
    for w, f, pf, pt in [(1, 8, 4, 2), (2, 4, 4, 2), (4, 32, 4, 2), (8, 16, 2, 2),
                         (4, 16, 1, 1), (16, 8, 4, 1), (3, 5, 4, 2)]:
        x = _rand_x(rng, w, f)
        g = _grid(mod, x, pf, pt)
        ref = np.fft.fft2(x, s=(pt * w, pf * f))
        assert g.shape == ref.shape
        assert np.allclose(g, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
        row0 = np.fft.fft(x.sum(axis=0), n=pf * f)
        assert np.allclose(g[0], row0, rtol=0, atol=1e-10 * np.abs(row0).max())


def check_parseval_and_energy(mod):
    """sum |G|^2 = M_t M_f sum |x|^2, and E (the mean power) = sum |x|^2 (P2)."""
    rng = np.random.default_rng(11)
    for w, f, pf, pt in [(4, 32, 4, 2), (1, 16, 4, 2), (8, 8, 2, 1)]:
        x = _rand_x(rng, w, f)
        g = _grid(mod, x, pf, pt)
        ex = float(np.sum(np.abs(x) ** 2))
        assert float(np.sum(np.abs(g) ** 2)) == pytest.approx(pt * w * pf * f * ex, rel=1e-12)
        r = mod.grid_peak(g)
        assert r.energy == pytest.approx(ex, rel=1e-12)


def check_on_grid_fringe(mod):
    """A unit fringe on grid bin (a, b) over all W APs peaks there with
    amplitude W*F and SNR sqrt(W*F) (P1 in general form)."""
    for w, f, pf, pt, a, b in [(4, 32, 4, 2, 3, 50), (8, 16, 4, 2, 13, 7),
                               (2, 64, 2, 2, 0, 100), (16, 8, 1, 1, 5, 3)]:
        mt, mf = pt * w, pf * f
        u = np.arange(w)[:, None]
        ff = np.arange(f)[None, :]
        x = np.exp(2j * np.pi * (a * u / mt + b * ff / mf))
        r = mod.search_window(x, 0, w, pf, pt)
        assert (r.k_rate, r.k_delay) == (a, b)
        assert r.amp == pytest.approx(w * f, rel=1e-12)
        assert r.snr == pytest.approx(math.sqrt(w * f), rel=1e-12)


def check_ties_and_zero(mod):
    """W = 1 rows are identical: the lower rate bin wins; an all-zero window
    gives peak (0, 0), amplitude 0, SNR 0."""
    rng = np.random.default_rng(3)
    x = _rand_x(rng, 1, 16)
    r = mod.search_window(x, 0, 1, 4, 2)
    assert r.k_rate == 0
    g = _grid(mod, x, 4, 2)
    assert np.array_equal(g[0], g[1])
    z = mod.search_window(np.zeros((4, 8), complex), 0, 4, 4, 2)
    assert (z.k_rate, z.k_delay, z.amp, z.snr, z.energy) == (0, 0, 0.0, 0.0, 0.0)


def check_window_counts(mod):
    """Window enumeration against the closed form floor((T-W)/s)+1 summed
    over lengths: 172132 per baseline for the EVN-like scan (T=58600,
    W=1..32) and 349761 for the large dense scan (T=117200, W=1..128)."""
    def closed(t, ws):
        return sum((t - w) // max(1, w // 2) + 1 for w in ws)
    for t, ws, expect in [(58600, [1, 2, 4, 8, 16, 32], 172132),
                          (117200, [1, 2, 4, 8, 16, 32, 64, 128], 349761),
                          (64, [4], 31)]:
        assert closed(t, ws) == expect
        assert sum(len(mod.window_starts(t, w)) for w in ws) == expect
    st = mod.window_starts(64, 4)
    assert st[0] == 0 and st[-1] == 60 and np.all(np.diff(st) == 2)
    assert list(mod.window_starts(5, 1)) == [0, 1, 2, 3, 4]
    assert len(mod.window_starts(3, 4)) == 0


def _c1_fringe_phasor_sum(t0, w):
    """sum of exp(i pi (t - 20) / 4) over the fringe APs 20..23 inside the
    window [t0, t0 + w): the 64-AP workload's fringe advances by half a rate
    bin (of 4 APs) per AP, i.e. by pi/4."""
    t = np.arange(max(t0, 20), min(t0 + w, 24))
    return complex(np.sum(np.exp(1j * np.pi * (t - 20) / 4)))


def check_delay_only_closed_form(mod):
    """Delay-only search of the noise-free 64-AP workload, from the closed
    form: the coherent sum of a window's fringe APs is 0.5 * C per channel
    (C = sum of the APs' phasors), on delay bin 13 exactly, so
    amp = F * 0.5 * |C|, E = F * 0.25 * |C|^2 and SNR = sqrt(F) = sqrt(32);
    windows without fringe APs are all-zero.  (The workload is stored in
    complex64, hence the 1e-6 tolerance.)"""
    spec = synth.c1(noise=False)
    v = spec.full()
    table, cands = mod.search_scan(v, [4], 4, 2, 3.0, spec.ap_seconds, spec.chan_width_hz,
                                   delay_only=True)
    assert len(table) == 31
    for row in table:
        c = _c1_fringe_phasor_sum(int(row["t_start"]), 4)
        assert row["k_rate"] == 0 and row["rate_hz"] == 0.0
        if abs(c) == 0.0:
            assert (row["k_delay"], row["amp"], row["snr"], row["energy"]) == (0, 0.0, 0.0, 0.0)
            continue
        assert row["k_delay"] == 13
        assert row["amp"] == pytest.approx(32 * 0.5 * abs(c), rel=1e-6)
        assert row["energy"] == pytest.approx(32 * 0.25 * abs(c) ** 2, rel=1e-6)
        assert row["snr"] == pytest.approx(math.sqrt(32), rel=1e-6)
    # windows 18, 20, 22 overlap the fringe; |C| = 2 cos(pi/8) for two APs,
    # |sin(pi/2) / sin(pi/8)| for all four
    assert [int(t) for t in cands["t_start"]] == [18, 20, 22]
    assert cands["amp"][1] == pytest.approx(16 / math.sin(math.pi / 8), rel=1e-6)
    assert cands["amp"][0] == pytest.approx(32 * math.cos(math.pi / 8), rel=1e-6)


def check_delay_only_library(mod):
    """The delay-only row equals numpy's FFT of the coherent AP sum, and the
    rate-0 row of the full grid; its mean power is sum_f |sum_u x|^2."""
    rng = np.random.default_rng(17)
    for w, f, pf in [(1, 8, 4), (2, 16, 4), (4, 32, 2), (8, 8, 1), (3, 5, 4)]:
        x = _rand_x(rng, w, f)
        row = mod.delay_only_row(x, pf)
        ref = np.fft.fft(x.sum(axis=0), n=pf * f)
        assert row.shape == (1, pf * f)
        assert np.allclose(row[0], ref, rtol=0, atol=1e-10 * np.abs(ref).max())
        r = mod.search_window_delay_only(x, 0, w, pf)
        assert r.energy == pytest.approx(float(np.sum(np.abs(x.sum(axis=0)) ** 2)), rel=1e-12)
        assert r.k_rate == 0 and r.k_delay == int(np.argmax(np.abs(ref) ** 2))


def check_delay_only_on_grid(mod):
    """A unit fringe on delay bin b with arbitrary per-AP phasors a_u peaks
    at b with amp = F |sum a_u| and SNR = sqrt(F) exactly."""
    rng = np.random.default_rng(23)
    for w, f, pf, b in [(4, 32, 4, 50), (8, 16, 2, 7), (2, 64, 1, 33)]:
        a = np.exp(2j * np.pi * rng.random(w)) * rng.uniform(0.5, 1.5, w)
        ff = np.arange(f)[None, :]
        x = a[:, None] * np.exp(2j * np.pi * b * ff / (pf * f))
        r = mod.search_window_delay_only(x, 0, w, pf)
        assert r.k_delay == b
        assert r.amp == pytest.approx(f * abs(a.sum()), rel=1e-12)
        assert r.snr == pytest.approx(math.sqrt(f), rel=1e-12)


def check_calibration(mod):
    """Gains that remove a per-channel instrumental delay put the fringe back
    on its true delay bin with amp = W*F and SNR = sqrt(W*F) (while the
    uncalibrated search peaks at the sum of both delays); flagged channels
    (gain 0) drop out of E (Parseval on the calibrated data); unit gains
    change nothing."""
    w, f, pf, pt, b_true, b_inst, a_rate = 4, 32, 4, 2, 21, 9, 3
    mt, mf = pt * w, pf * f
    u = np.arange(w)[:, None]
    ff = np.arange(f)[None, :]
    x = np.exp(2j * np.pi * (a_rate * u / mt + (b_true + b_inst) * ff / mf))
    vis = x[None]                                  # one baseline
    g = np.exp(-2j * np.pi * b_inst * np.arange(f) / mf)[None, :]
    t_raw, _ = mod.search_scan(vis, [w], pf, pt, 1.0, 1.0, 1.0)
    t_cal, _ = mod.search_scan(vis, [w], pf, pt, 1.0, 1.0, 1.0, gains=g)
    assert (t_raw["k_rate"][0], t_raw["k_delay"][0]) == (a_rate, b_true + b_inst)
    assert (t_cal["k_rate"][0], t_cal["k_delay"][0]) == (a_rate, b_true)
    assert t_cal["amp"][0] == pytest.approx(w * f, rel=1e-12)
    assert t_cal["snr"][0] == pytest.approx(math.sqrt(w * f), rel=1e-12)
    rng = np.random.default_rng(29)
    xr = _rand_x(rng, 6, f)[None]
    mask = np.ones((1, f))
    mask[0, 5:17] = 0.0
    t_m, _ = mod.search_scan(xr, [2], pf, pt, 1.0, 1.0, 1.0, gains=mask)
    e_want = [float(np.sum(np.abs(xr[0, t0:t0 + 2, mask[0] > 0]) ** 2)) for t0 in range(5)]
    assert np.allclose(t_m["energy"], e_want, rtol=1e-12)
    t_1, _ = mod.search_scan(xr, [2], pf, pt, 1.0, 1.0, 1.0, gains=np.ones((1, f)))
    t_0, _ = mod.search_scan(xr, [2], pf, pt, 1.0, 1.0, 1.0)
    assert np.array_equal(t_1, t_0)


def check_autospectrum_normalization(mod):
    """A fringe seen through the stations' bandpasses B_i(f) (cross
    spectrum B_i B_j x, auto-spectra a_i = B_i^2) is flattened by the
    normalisation, so the closed form of an on-grid fringe holds again:
    amp = W*F, SNR = sqrt(W*F) on every baseline (the raw search falls
    short of that SNR).  Auto-spectra that vary over time enter through the
    mean of their squares: uniform ones scale amp by
    (abar_i^2 abar_j^2)^(-1/4) and leave the SNR and the bins.  A station
    with a zero auto-spectrum channel flags that channel."""
    w, f, pf, pt, kt, kf = 4, 32, 4, 2, 3, 17
    mt, mf = pt * w, pf * f
    rng = np.random.default_rng(41)
    pairs = [(0, 1), (0, 2), (1, 2)]
    bp = rng.uniform(0.3, 2.0, (3, f))
    u = np.arange(w)[:, None]
    ff = np.arange(f)[None, :]
    fr = np.exp(2j * np.pi * (kt * u / mt + kf * ff / mf))
    vis = np.stack([bp[i] * bp[j] * fr for i, j in pairs])
    auto = np.repeat((bp ** 2)[:, None, :], 5, axis=1)
    g = mod.autospectrum_gains(auto, pairs)
    t, _ = mod.search_scan(vis, [w], pf, pt, 1.0, 1.0, 1.0, gains=g)
    t_raw, _ = mod.search_scan(vis, [w], pf, pt, 1.0, 1.0, 1.0)
    for b in range(3):
        assert (t["k_rate"][b], t["k_delay"][b]) == (kt, kf)
        assert t["amp"][b] == pytest.approx(w * f, rel=1e-12)
        assert t["snr"][b] == pytest.approx(math.sqrt(w * f), rel=1e-12)
        assert t_raw["snr"][b] < 0.99 * math.sqrt(w * f)
    # uniform auto-spectra varying over time: station 0 alternates c1, c2
    c1, c2, d = 0.5, 2.0, 1.5
    a2 = np.empty((2, 4, f))
    a2[0, 0::2], a2[0, 1::2], a2[1] = c1, c2, d
    xr = _rand_x(rng, 8, f)[None]
    g2 = mod.autospectrum_gains(a2, [(0, 1)])
    want = (((c1 ** 2 + c2 ** 2) / 2) * d ** 2) ** -0.25
    assert np.allclose(g2, want, rtol=1e-14)
    t2, _ = mod.search_scan(xr, [2, 4], pf, pt, 1.0, 1.0, 1.0, gains=g2)
    t0_, _ = mod.search_scan(xr, [2, 4], pf, pt, 1.0, 1.0, 1.0)
    assert np.array_equal(t2["k_rate"], t0_["k_rate"]) and np.array_equal(t2["k_delay"], t0_["k_delay"])
    assert np.allclose(t2["amp"], want * t0_["amp"], rtol=1e-12)
    assert np.allclose(t2["snr"], t0_["snr"], rtol=1e-12)
    # a zero auto-spectrum channel of either station flags it on the baseline
    a3 = np.ones((2, 3, f))
    a3[1, :, 7] = 0.0
    g3 = mod.autospectrum_gains(a3, [(0, 1), (0, 0)])
    assert g3[0, 7] == 0.0 and np.all(np.delete(g3[0], 7) == 1.0) and np.all(g3[1] == 1.0)


def check_dedispersion(mod):
    """A unit pulse that reaches channel f at AP t0 + d_f (dispersed) is
    restored by the shifts d_f: the one-AP window at t0 then holds every
    channel, amp = F and SNR = sqrt(F) at delay bin 0, and the APs after it
    are empty; with zero shifts the search is unchanged."""
    f, t, t0 = 32, 40, 5
    d = (np.arange(f)[::-1] * 3) // 4          # 0 .. 23 APs, larger at low f
    vis = np.zeros((1, t, f), complex)
    vis[0, t0 + d, np.arange(f)] = 1.0
    tab, _ = mod.search_scan(vis, [1], 4, 2, 1.0, 1.0, 1.0, shifts=d)
    r = tab[tab["t_start"] == t0][0]
    assert (r["k_rate"], r["k_delay"]) == (0, 0)
    assert r["amp"] == pytest.approx(f, rel=1e-12)
    assert r["snr"] == pytest.approx(math.sqrt(f), rel=1e-12)
    assert np.all(tab[tab["t_start"] != t0]["amp"] == 0.0)
    raw, _ = mod.search_scan(vis, [1], 4, 2, 1.0, 1.0, 1.0)
    # undispersed, the window at t0 holds only the channels with no delay
    assert raw[raw["t_start"] == t0]["amp"][0] == pytest.approx(float(np.sum(d == 0)), rel=1e-12)
    rng = np.random.default_rng(31)
    xr = _rand_x(rng, 9, 16)[None]
    z, _ = mod.search_scan(xr, [1, 4], 4, 2, 1.0, 1.0, 1.0, shifts=np.zeros(16, int))
    n, _ = mod.search_scan(xr, [1, 4], 4, 2, 1.0, 1.0, 1.0)
    assert np.array_equal(z, n)


ALL_CHECKS = [check_c1_closed_form, check_library_fft, check_parseval_and_energy,
              check_on_grid_fringe, check_ties_and_zero, check_window_counts,
              check_delay_only_closed_form, check_delay_only_library, check_delay_only_on_grid,
              check_calibration, check_autospectrum_normalization, check_dedispersion]


@pytest.mark.parametrize("check", ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(check):
    check(fo)


# ---------------------------------------------------- statistical laws -----

def test_noise_bin_law():
    """Noise only: at a fixed bin, SNR^2 / N ~ Beta(1, N-1), N = W*F, for any
    padding (P5).  KS over 2000 seeds."""
    w, f, pf, pt = 2, 4, 4, 2
    n = w * f
    vals = []
    for s in range(2000):
        x = _rand_x(np.random.default_rng([123, s]), w, f)
        g = _grid(fo, x, pf, pt)
        e = fo.grid_peak(g).energy
        vals.append(abs(g[1, 3]) ** 2 / e / n)
    p = stats.kstest(vals, stats.beta(1, n - 1).cdf).pvalue
    assert p > 1e-3


def _fisher_g_sf(x, m):
    j = np.arange(1, int(math.floor(1.0 / x)) + 1)
    return float(np.sum((-1.0) ** (j - 1) * special.comb(m, j) * (1 - j * x) ** (m - 1)))


def test_noise_max_fisher_g():
    """Noise only, unpadded grid: SNR_max^2 / M follows Fisher's g for M
    complex ordinates (P6).  KS over 2000 seeds."""
    w, f = 2, 4
    m = w * f
    gs = []
    for s in range(2000):
        x = _rand_x(np.random.default_rng([321, s]), w, f)
        r = fo.search_window(x, 0, w, 1, 1)
        gs.append(r.snr ** 2 / m)
    p = stats.kstest(gs, lambda v: np.array([1.0 - _fisher_g_sf(t, m) if t > 0 else 0.0
                                             for t in np.atleast_1d(v)])).pvalue
    assert p > 1e-3


def test_delay_only_noise_laws():
    """Noise only, delay-only search: at a fixed delay bin SNR^2 / F ~
    Beta(1, F-1) for any padding and window length (the coherent sum of W
    complex Gaussian APs is again one), and unpadded the maximum follows
    Fisher's g for F ordinates.  KS over 2000 seeds each."""
    w, f = 3, 8
    bins, maxes = [], []
    for s in range(2000):
        x = _rand_x(np.random.default_rng([456, s]), w, f)
        row = fo.delay_only_row(x, 4)[0]
        e = float(np.mean(np.abs(row) ** 2))
        bins.append(abs(row[5]) ** 2 / e / f)
        r = fo.search_window_delay_only(x, 0, w, 1)
        maxes.append(r.snr ** 2 / f)
    assert stats.kstest(bins, stats.beta(1, f - 1).cdf).pvalue > 1e-3
    p = stats.kstest(maxes, lambda v: np.array([1.0 - _fisher_g_sf(t, f) if t > 0 else 0.0
                                                for t in np.atleast_1d(v)])).pvalue
    assert p > 1e-3


# ---------------------------------------------------------- invariances ----

def test_shift_invariance():
    """x * exp(+2 pi i (a u / M_t + b f / M_f)) moves the peak by (a, b) (P8)."""
    rng = np.random.default_rng(5)
    w, f, pf, pt = 8, 16, 4, 2
    mt, mf = pt * w, pf * f
    x = _rand_x(rng, w, f)
    r0 = fo.search_window(x, 0, w, pf, pt)
    for a, b in [(1, 0), (0, 1), (5, 40), (15, 63)]:
        u = np.arange(w)[:, None]
        ff = np.arange(f)[None, :]
        xs = x * np.exp(2j * np.pi * (a * u / mt + b * ff / mf))
        r = fo.search_window(xs, 0, w, pf, pt)
        assert (r.k_rate, r.k_delay) == ((r0.k_rate + a) % mt, (r0.k_delay + b) % mf)
        assert r.amp == pytest.approx(r0.amp, rel=1e-12)
        assert r.snr == pytest.approx(r0.snr, rel=1e-12)


def test_scale_invariance():
    """x -> c x keeps the peak and SNR, scales amp by |c| (P9)."""
    rng = np.random.default_rng(9)
    x = _rand_x(rng, 4, 32)
    r0 = fo.search_window(x, 0, 4, 4, 2)
    c = 3.7 * np.exp(1j * 0.3)
    r = fo.search_window(c * x, 0, 4, 4, 2)
    assert (r.k_rate, r.k_delay) == (r0.k_rate, r0.k_delay)
    assert r.snr == pytest.approx(r0.snr, rel=1e-12)
    assert r.amp == pytest.approx(abs(c) * r0.amp, rel=1e-12)


def test_partial_overlap():
    """A fringe over q of the W APs at an on-grid rate peaks at a*q*F (P10)."""
    w, f, pf, pt = 8, 16, 4, 2
    mt, mf = pt * w, pf * f
    for q, first in [(3, 0), (5, 3), (1, 7)]:
        x = np.zeros((w, f), complex)
        u = np.arange(first, first + q)[:, None]
        ff = np.arange(f)[None, :]
        x[first:first + q] = 0.25 * np.exp(2j * np.pi * (2 * u / mt + 9 * ff / mf))
        r = fo.search_window(x, 0, w, pf, pt)
        # one AP is flat across rate bins: the tie goes to rate bin 0
        assert (r.k_rate, r.k_delay) == ((2 if q > 1 else 0), 9)
        assert r.amp == pytest.approx(0.25 * q * f, rel=1e-12)
        assert r.snr == pytest.approx(math.sqrt(q * f), rel=1e-12)


def test_signed_bins_and_units():
    assert fo.signed_bin(0, 8) == 0 and fo.signed_bin(3, 8) == 3
    assert fo.signed_bin(4, 8) == -4 and fo.signed_bin(7, 8) == -1
    spec = synth.c1(noise=False)
    _, c = fo.search_scan(spec.full(), [4], 4, 2, 3.0, spec.ap_seconds, spec.chan_width_hz)
    # k_f = 13 of 128 bins, df = 1/32: tau = 13 / (128 / 32) = 3.25 (the injected delay)
    assert c["delay_s"][1] == pytest.approx(3.25)
    # k_t = 1 of 8 bins, T_ap = 1: nu = 1/8 (the injected rate)
    assert c["rate_hz"][1] == pytest.approx(0.125)


def test_generator_determinism():
    """Any baseline regenerates alone, bit for bit; the threaded full scan
    equals the per-baseline arrays."""
    spec = synth.c2(n_stations=4, n_ap=300)
    full = spec.full(threads=3)
    for b in range(spec.n_baselines):
        assert np.array_equal(full[b], spec.baseline(b))
    assert np.array_equal(spec.baseline(2, 100, 140), full[2, 100:140])


# ------------------------------------------------------ planted mistakes ---

def _mutant(**overrides):
    m = types.ModuleType("mutant_oracle")
    m.__dict__.update({k: getattr(fo, k) for k in dir(fo) if not k.startswith("__")})
    m.__dict__.update(overrides)
    # rebind functions so their globals see the overrides
    for name in ("delay_spectra", "window_grid", "search_window", "search_baseline",
                 "search_scan", "window_starts", "grid_peak", "delay_only_row",
                 "search_window_delay_only", "calibrate", "dedisperse",
                 "autospectrum_gains"):
        f = getattr(fo, name)
        if name in overrides:
            continue
        g = types.FunctionType(f.__code__, m.__dict__, name, f.__defaults__, f.__closure__)
        setattr(m, name, g)
    return m


def _fails(mod):
    for c in ALL_CHECKS:
        try:
            c(mod)
        except AssertionError:
            return True
    return False


def _flip_sign_delay(n_freq, m_f):
    return np.conj(fo.delay_dft_matrix(n_freq, m_f))


def _rate_no_pad(window_ap, m_t):
    return fo.rate_dft_matrix(window_ap, window_ap)[:, :] if m_t == window_ap else \
        np.vstack([fo.rate_dft_matrix(window_ap, window_ap)] * (m_t // window_ap))


def _peak_sum_energy(g, duplicate_rate_rows=False):
    r = fo.grid_peak(g, duplicate_rate_rows)
    e = r.energy * g.size
    r.energy = e
    r.snr = r.amp / math.sqrt(e) if e > 0 else 0.0
    return r


def _peak_last_tie(g, duplicate_rate_rows=False):
    p = np.abs(g) ** 2
    flat = p.size - 1 - int(np.argmax(p.ravel()[::-1]))
    r = fo.grid_peak(g, duplicate_rate_rows)
    r.k_rate, r.k_delay = divmod(flat, p.shape[1])
    return r


def _starts_full_stride(n_ap, w):
    return np.arange(0, n_ap - w + 1, w) if n_ap >= w else np.zeros(0, int)


def _transposed_freq(x_b, pad_freq):
    x_b = np.asarray(x_b, complex)
    # IF-major mistake: channel and IF axes swapped inside each AP
    t, f = x_b.shape
    return fo.delay_spectra(x_b.reshape(t, 2, f // 2).transpose(0, 2, 1).reshape(t, f), pad_freq)


def _delay_only_incoherent(x_seg, pad_freq, a_f=None):
    # per-AP power spectra summed (an incoherent search), not the coherent sum
    x_seg = np.asarray(x_seg, complex)
    spec = x_seg @ fo.delay_dft_matrix(x_seg.shape[1], pad_freq * x_seg.shape[1])
    return np.sqrt(np.sum(np.abs(spec) ** 2, axis=0))[None, :].astype(complex)


def _delay_only_grid_energy(x_b, t0, window_ap, pad_freq, a_f=None):
    # E taken as the full grid's (sum of |x|^2) instead of the delay row's
    r = fo.search_window_delay_only(x_b, t0, window_ap, pad_freq, a_f)
    e = float(np.sum(np.abs(np.asarray(x_b[t0:t0 + window_ap])) ** 2))
    r.energy = e
    r.snr = r.amp / math.sqrt(e) if e > 0 else 0.0
    return r


def _dedisperse_backwards(vis, shifts):
    # channels moved later instead of earlier
    vis = np.asarray(vis, complex)
    out = np.zeros_like(vis)
    for f, k in enumerate(np.asarray(shifts, int)):
        if k < vis.shape[1]:
            out[:, k:, f] = vis[:, :vis.shape[1] - k, f]
    return out


def _calibrate_conjugate(vis, gains):
    # the conjugate gains: adds the instrumental delay instead of removing it
    return fo.calibrate(vis, np.conj(np.asarray(gains)))


def _auto_half_power(auto, pairs):
    # (abar_i^2 abar_j^2)^(-1/2): the exponent of a power, not an amplitude
    return fo.autospectrum_gains(auto, pairs) ** 2


def _auto_mean_then_square(auto, pairs):
    # the square of the mean auto-spectrum instead of the mean of its squares
    a = np.asarray(auto, float)
    m = a.mean(axis=1, keepdims=True)
    return fo.autospectrum_gains(np.repeat(m, a.shape[1], axis=1), pairs)


def _auto_one_station(auto, pairs):
    # the first station's dispersion taken twice
    return fo.autospectrum_gains(auto, [(i, i) for i, _ in pairs])


@pytest.mark.parametrize("overrides", [
    dict(autospectrum_gains=_auto_half_power),
    dict(autospectrum_gains=_auto_mean_then_square),
    dict(autospectrum_gains=_auto_one_station),
    dict(calibrate=_calibrate_conjugate),
    dict(dedisperse=_dedisperse_backwards),
    dict(delay_only_row=_delay_only_incoherent),
    dict(search_window_delay_only=_delay_only_grid_energy),
    dict(delay_dft_matrix=_flip_sign_delay),
    dict(rate_dft_matrix=_rate_no_pad),
    dict(grid_peak=_peak_sum_energy),
    dict(grid_peak=_peak_last_tie),
    dict(window_starts=_starts_full_stride),
    dict(delay_spectra=_transposed_freq),
], ids=["autospectrum-half-power", "autospectrum-mean-then-square", "autospectrum-one-station",
        "calibration-conjugate", "dedispersion-backwards", "delay-only-incoherent", "delay-only-grid-energy", "delay-sign", "rate-pad",
        "energy-sum", "tie-last", "stride", "freq-order"])
def test_planted_mistake_is_caught(overrides):
    assert _fails(_mutant(**overrides))


def test_unmutated_reference_passes_all_checks():
    assert not _fails(fo)
