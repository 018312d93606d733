"""Parity of the library's candidate consumers (host code behind the C ABI:
fringe_match, fringe_localize, fringe_delay_partials) with the reference
matching and localization, on the same seeded inputs.  Matching is integer
and selection work: rows must be identical field by field.  Localization is
FP64 least squares by a different factorisation: 1e-9 relative (the fits
here have condition numbers below 1e3, so rounding stays near 1e-13)."""

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import oracle.pulse_match_oracle as pm
import paper_2108_05602_amd as F
import synth
from paper_2108_05602_amd import binding as B


def _oracle_rows(cands, min_windows, min_baselines):
    rows = pm.single_pulses(cands, min_windows, min_baselines)
    out = np.zeros(len(rows), B.PULSE_DTYPE)
    for i, r in enumerate(rows):
        for k in pm.PULSE_FIELDS:
            out[i][k] = r[k]
    return out


def _same(got, ref):
    assert len(got) == len(ref)
    for k in pm.PULSE_FIELDS:
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("seed,min_windows,min_baselines", [
    (1, 2, 5), (2, 2, 5), (3, 1, 1), (4, 3, 8), (5, 2, 2)])
def test_match_random_lists(seed, min_windows, min_baselines):
    c = synth.candidate_list(seed, n_scans=2, n_baselines=21, n_ap=6000, n_pulses=12,
                             n_noise=800)
    got, n_p = F.fringe_match(c, min_windows, min_baselines)
    ref = _oracle_rows(c, min_windows, min_baselines)
    _same(got, ref)
    assert n_p == len(set(ref["pulse"].tolist()))


def test_match_is_order_independent_and_reports_capacity():
    c = synth.candidate_list(9, n_scans=2, n_baselines=10, n_ap=3000, n_pulses=6, n_noise=100)
    a, na = F.fringe_match(c)
    b, nb = F.fringe_match(c[::-1].copy())
    assert na == nb and a.tobytes() == b.tobytes() and na > 0
    lib = F.load()
    import ctypes
    p = B.fringe_match_params(2, 5)
    out = np.zeros(3, B.PULSE_DTYPE)
    nr, npl = ctypes.c_int64(0), ctypes.c_int64(0)
    cc = B.as_candidates(c)
    rc = lib.fringe_match(cc.ctypes.data_as(ctypes.c_void_p), len(cc), ctypes.byref(p),
                          out.ctypes.data_as(ctypes.c_void_p), 3, ctypes.byref(nr),
                          ctypes.byref(npl))
    assert rc == B.FRINGE_E_CAPACITY and nr.value == len(a) and npl.value == na
    assert out.tobytes() == a[:3].tobytes()


def test_match_edge_cases():
    empty = np.zeros(0, B.CANDIDATE_DTYPE)
    rows, n = F.fringe_match(empty)
    assert len(rows) == 0 and n == 0
    one = np.zeros(1, B.CANDIDATE_DTYPE)
    one[0] = (0, 0, 4, 0, 0, 0, 1.0, 5.0, 1.0, 0, 0.0, 0.0)
    rows, n = F.fringe_match(one, 1, 1)
    assert n == 1 and rows[0]["t_lo"] == 0 and rows[0]["t_hi"] == 4
    for bad in [dict(window_ap=0), dict(t_start=-1), dict(snr=np.nan)]:
        c = one.copy()
        for k, v in bad.items():
            c[0][k] = v
        with pytest.raises(F.FringeError) as e:
            F.fringe_match(c, 1, 1)
        assert e.value.code == B.FRINGE_E_INVALID
    with pytest.raises(F.FringeError):
        F.fringe_match(one, 0, 1)


def test_match_on_searched_scan():
    """A small EVN-like scan (6 stations, 1500 APs, 4 pulses, 2 RFI tones
    that last the whole scan) searched by the reference: both matchers agree,
    every planted pulse is found as exactly one single pulse, and the tones
    do not chain the pulses together."""
    spec = synth.c2(seed=21, n_stations=6, n_ap=1500, n_pulses=4, n_tones=2)
    vis = spec.full(threads=4)
    tab, cands = fo.search_scan(vis, [1, 2, 4, 8, 16, 32], 4, 2, 4.5, spec.ap_seconds,
                                spec.chan_width_hz)
    cands = B.as_candidates(cands)       # the records as the library holds them
    got, n_p = F.fringe_match(cands, 2, 5)
    _same(got, _oracle_rows(cands, 2, 5))
    assert n_p == len(spec.pulses) == 4
    for p in spec.pulses:
        hit = {int(r["pulse"]) for r in got if r["t_lo"] < p.start + p.width and p.start < r["t_hi"]}
        assert len(hit) == 1, (p.start, p.width, p.snr, hit)


def test_localize_parity():
    rng = np.random.default_rng(17)
    for n in (2, 3, 5, 12, 45):
        a = rng.normal(0, 1e-4, n)
        d = rng.normal(0, 1e-4, n)
        tau = rng.normal(0, 1e-10, n) + 3e-6 * a - 1e-6 * d
        sol, rms, loo, loo_rms = F.fringe_localize(tau, a, d)
        rs, rr, rl, rlr = pm.localize(tau, a, d)
        np.testing.assert_allclose(sol, rs, rtol=1e-9, atol=0)
        assert abs(rms - rr) <= 1e-9 * rr + 1e-12 * np.max(np.abs(tau))
        assert loo.shape == rl.shape and len(loo_rms) == len(rlr)
        np.testing.assert_allclose(loo, rl, rtol=1e-9, atol=0)
        np.testing.assert_allclose(loo_rms, rlr, rtol=1e-9, atol=1e-12 * np.max(np.abs(tau)))


def test_localize_errors_and_degenerate_subsets():
    with pytest.raises(F.FringeError):
        F.fringe_localize([1e-9], [1e-4], [2e-4])
    with pytest.raises(F.FringeError):
        F.fringe_localize([1e-9, 2e-9, 0], [1e-4, 2e-4, 3e-4], [2e-4, 4e-4, 6e-4])
    with pytest.raises(F.FringeError):
        F.fringe_localize([1e-9, np.inf, 0], [1e-4, 2e-4, 3e-4], [1e-4, 0, 1e-4])
    # the only baseline with a dec partial left out: that solve is undefined
    a = np.array([1e-4, 2e-4, 3e-4])
    d = np.array([0.0, 0.0, 1e-4])
    tau = 2e-6 * a + 5e-6 * d
    sol, rms, loo, loo_rms = F.fringe_localize(tau, a, d)
    np.testing.assert_allclose(sol, [2e-6, 5e-6], rtol=1e-12)
    assert np.all(np.isnan(loo[2])) and np.isnan(loo_rms[2])
    np.testing.assert_allclose(loo[:2], [[2e-6, 5e-6]] * 2, rtol=1e-12)


def test_delay_partials_parity():
    rng = np.random.default_rng(2)
    b = rng.normal(0, 4e6, (45, 3))
    for gast, ra, dec in [(0.3, 1.2, 0.4), (5.9, 0.1, -0.9), (2.0, 2.0, 1.5707963267948966)]:
        da, dd = F.fringe_delay_partials(b, gast, ra, dec)
        ra_, rd_ = pm.delay_partials(b, gast, ra, dec)
        scale = np.linalg.norm(b, axis=1) / pm.C_LIGHT
        assert np.all(np.abs(da - ra_) <= 1e-14 * scale)
        assert np.all(np.abs(dd - rd_) <= 1e-14 * scale)
    da, dd = F.fringe_delay_partials(np.zeros((0, 3)), 0.0, 0.0, 0.0)
    assert len(da) == 0 and len(dd) == 0
