"""Pins of the reference single-pulse matching and localization: hand-built
candidate lists whose pulses follow from the criteria by inspection, and
localization recovering a known offset exactly and singling out a corrupted
baseline.  Planted mistakes in the reference must fail one of the checks."""

import types

import numpy as np
import pytest

import oracle.pulse_match_oracle as pm
from oracle.fringe_oracle import TABLE_DTYPE


def _c(rows):
    out = np.zeros(len(rows), TABLE_DTYPE)
    for i, (scan, b, w, t, snr) in enumerate(rows):
        out[i]["scan"], out[i]["baseline"], out[i]["window_ap"], out[i]["t_start"] = scan, b, w, t
        # amp falls as SNR rises, so a representative chosen by amp is caught
        out[i]["snr"], out[i]["amp"] = snr, 100.0 - snr
        out[i]["k_delay"], out[i]["delay_s"] = b + 1, 1e-9 * (b + 1)
    return out


def check_baseline_pulses(mod):
    rows = [
        (0, 0, 2, 10, 5.0), (0, 0, 4, 9, 6.0),                      # two lengths overlap: pulse
        (0, 0, 2, 40, 7.0), (0, 0, 2, 41, 8.0),                     # one length only: none
        (0, 0, 2, 60, 5.0), (0, 0, 8, 61, 5.0), (0, 0, 2, 68, 9.0), # 60-62 does not touch the
                                                                    # anchor 68-70: left alone
        (0, 1, 2, 10, 5.0), (0, 1, 4, 12, 5.0),                     # touching, no shared AP: none
    ]
    ps = sorted(mod.baseline_pulses(_c(rows), min_windows=2), key=lambda p: (p["baseline"], p["t_lo"]))
    got = [(p["baseline"], p["t_lo"], p["t_hi"], p["n_windows"], p["n_lengths"],
            int(p["rep"]["t_start"])) for p in ps]
    assert got == [(0, 9, 13, 2, 2, 9), (0, 61, 70, 2, 2, 68)]
    # SNR ties: the shorter window, then the earlier start, anchors the group
    ps = mod.baseline_pulses(_c([(0, 3, 4, 20, 5.0), (0, 3, 2, 21, 5.0), (0, 3, 2, 23, 5.0)]))
    assert [(int(p["rep"]["window_ap"]), int(p["rep"]["t_start"]), p["n_windows"]) for p in ps] \
        == [(2, 21, 2)]


def check_single_pulses(mod):
    # baseline pulses on 6 baselines around AP 100; baseline 5's is apart (AP 300)
    rows = []
    for b in range(6):
        t = 100 + b // 2 if b < 5 else 300
        rows += [(0, b, 2, t, 5.0 + b), (0, b, 4, t - 1, 4.0)]
    sp = mod.single_pulses(_c(rows), min_windows=2, min_baselines=5)
    assert [r["baseline"] for r in sp] == [0, 1, 2, 3, 4]
    assert {r["pulse"] for r in sp} == {0}
    assert all(r["window_ap"] == 2 and r["t_start"] == 100 + r["baseline"] // 2 for r in sp)
    assert [(r["t_lo"], r["t_hi"]) for r in sp] == [(99 + b // 2, 103 + b // 2) for b in range(5)]
    assert mod.single_pulses(_c(rows), min_windows=2, min_baselines=6) == []
    # a second scan is matched on its own, and numbered after the first
    rows2 = rows + [(1, b, 2, 100, 5.0) for b in range(5)] + [(1, b, 8, 98, 5.0) for b in range(5)]
    sp2 = mod.single_pulses(_c(rows2), min_windows=2, min_baselines=5)
    assert [(r["scan"], r["pulse"]) for r in sp2] == [(0, 0)] * 5 + [(1, 1)] * 5
    # a group of five baseline pulses on four baselines (baseline 0 has two,
    # both touching the anchor on baseline 1): no single pulse at five; at
    # four, baseline 0 is represented by its stronger pulse
    rows3 = [(0, 1, 16, 40, 9.0), (0, 1, 8, 44, 3.0),
             (0, 0, 2, 42, 6.0), (0, 0, 4, 41, 1.0), (0, 0, 2, 50, 7.0), (0, 0, 4, 49, 1.0)]
    for b in (2, 3):
        rows3 += [(0, b, 8, 48, 5.0), (0, b, 4, 52, 5.0)]
    assert mod.single_pulses(_c(rows3), min_windows=2, min_baselines=5) == []
    sp3 = mod.single_pulses(_c(rows3), min_windows=2, min_baselines=4)
    assert [r["baseline"] for r in sp3] == [0, 1, 2, 3]
    assert (sp3[0]["t_start"], sp3[0]["snr"], sp3[0]["t_lo"]) == (50, 7.0, 49)
    assert (sp3[1]["t_lo"], sp3[1]["t_hi"], sp3[2]["t_start"]) == (40, 56, 52)
    # equal SNR and window: the earlier start; input order does not matter
    rows4 = rows3[:4] + [(0, 0, 2, 50, 6.0)] + rows3[5:]
    rows4 = rows4[3:] + rows4[:3]
    sp4 = mod.single_pulses(_c(rows4), min_windows=2, min_baselines=4)
    assert (sp4[0]["t_start"], sp4[0]["t_lo"]) == (42, 41)
    # a long-lived signal on one baseline does not chain two pulses together
    rows5 = [(0, 9, 32, t, 4.6) for t in range(0, 400, 16)] + \
            [(0, 9, 16, t, 4.6) for t in range(0, 400, 8)]
    for b in range(5):
        rows5 += [(0, b, 2, 100, 8.0), (0, b, 4, 99, 6.0), (0, b, 2, 300, 8.0), (0, b, 4, 299, 6.0)]
    sp5 = mod.single_pulses(_c(rows5), min_windows=2, min_baselines=5)
    assert sorted({(r["pulse"], r["t_lo"]) for r in sp5 if r["baseline"] == 0}) == [(0, 99), (1, 299)]


def check_localize(mod):
    rng = np.random.default_rng(3)
    n = 7
    a = rng.normal(0, 1e-4, n)     # s/rad partials
    d = rng.normal(0, 1e-4, n)
    truth = np.array([2.5e-6, -1.2e-6])
    tau = a * truth[0] + d * truth[1]
    sol, rms, loo, loo_rms = mod.localize(tau, a, d)
    assert np.allclose(sol, truth, rtol=1e-9, atol=0) and rms < 1e-20
    assert loo.shape == (n, 2) and np.allclose(loo, truth, rtol=1e-9, atol=0)
    assert np.all(loo_rms < 1e-20)
    # a corrupted baseline: only the fit without it is exact again
    bad = tau.copy()
    bad[4] += 3e-10
    sol, rms, loo, loo_rms = mod.localize(bad, a, d)
    assert int(np.argmin(loo_rms)) == 4 and loo_rms[4] < 1e-20
    assert np.all(np.delete(loo_rms, 4) > 1e-12) and rms > 1e-12
    assert np.allclose(loo[4], truth, rtol=1e-9, atol=0)
    assert not np.allclose(sol, truth, rtol=1e-3, atol=0)
    # two baselines: a 2x2 solve, no leave-one-out
    sol, rms, loo, loo_rms = mod.localize(tau[:2], a[:2], d[:2])
    assert np.allclose(sol, truth, rtol=1e-9, atol=0) and loo.shape == (0, 2) and len(loo_rms) == 0




# ------------------------------------------------------ delay partials ---

def _tau_by_rotation(b, gast, ra, dec):
    # the source's celestial unit vector turned into the Earth-fixed frame by
    # a rotation of -gast about the pole; tau_g = -(b . s) / c
    s_cel = np.array([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)])
    c, s = np.cos(gast), np.sin(gast)
    rot = np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])
    return -(np.asarray(b, float) @ (rot @ s_cel)) / pm.C_LIGHT


def check_delay_partials(mod):
    rng = np.random.default_rng(11)
    b = rng.normal(0, 3e6, (9, 3))
    for gast, ra, dec in [(1.1, 0.9, 0.3), (4.0, 5.5, -1.2), (0.2, 3.0, 1.5)]:
        da, dd = mod.delay_partials(b, gast, ra, dec)
        h = 1e-6
        fa = (_tau_by_rotation(b, gast, ra + h, dec) - _tau_by_rotation(b, gast, ra - h, dec)) / (2 * h)
        fd = (_tau_by_rotation(b, gast, ra, dec + h) - _tau_by_rotation(b, gast, ra, dec - h)) / (2 * h)
        scale = np.linalg.norm(b, axis=1) / pm.C_LIGHT
        assert np.all(np.abs(da - fa) < 1e-7 * scale) and np.all(np.abs(dd - fd) < 1e-7 * scale)
    # at the pole the delay does not depend on ra; a polar baseline sees no ra term
    da, dd = mod.delay_partials(b, 0.7, 1.3, np.pi / 2)
    assert np.all(np.abs(da) < 1e-16 * np.linalg.norm(b, axis=1))
    da, _ = mod.delay_partials([[0.0, 0.0, 6e6]], 0.7, 1.3, 0.4)
    assert da[0] == 0.0
    # reversing a baseline reverses its partials
    da1, dd1 = mod.delay_partials(b, 2.0, 1.0, 0.5)
    da2, dd2 = mod.delay_partials(-b, 2.0, 1.0, 0.5)
    assert np.array_equal(da1, -da2) and np.array_equal(dd1, -dd2)


def check_localize_geometric(mod):
    # an offset source: the delay residuals against the a priori position,
    # fitted with the partials, recover the offset to first order
    rng = np.random.default_rng(5)
    st = rng.normal(0, 3e6, (6, 3))
    b = np.array([st[j] - st[i] for i in range(6) for j in range(i + 1, 6)])
    gast, ra0, dec0 = 1.7, 0.8, 0.6
    off = np.array([2e-7, -3e-7])          # rad (~0.04", -0.06")
    tau = _tau_by_rotation(b, gast, ra0 + off[0], dec0 + off[1]) - _tau_by_rotation(b, gast, ra0, dec0)
    da, dd = mod.delay_partials(b, gast, ra0, dec0)
    sol, rms, _, _ = mod.localize(tau, da, dd)
    assert np.allclose(sol, off, rtol=1e-5, atol=0)


ALL_CHECKS = [check_baseline_pulses, check_single_pulses, check_localize, check_delay_partials,
              check_localize_geometric]


@pytest.mark.parametrize("check", ALL_CHECKS, ids=lambda c: c.__name__)
def test_reference_matching(check):
    check(pm)


# ------------------------------------------------------ planted mistakes ---

def _mutant(**overrides):
    m = types.ModuleType("mutant_match")
    m.__dict__.update({k: getattr(pm, k) for k in dir(pm) if not k.startswith("__")})
    m.__dict__.update(overrides)
    for name in ("baseline_pulses", "single_pulses", "localize", "_anchored_groups",
                 "_window_strength", "_pulse_strength", "delay_partials"):
        if name in overrides:
            continue
        f = getattr(pm, name)
        setattr(m, name, types.FunctionType(f.__code__, m.__dict__, name, f.__defaults__,
                                            f.__closure__))
    return m


def _fails(mod):
    for c in ALL_CHECKS:
        try:
            c(mod)
        except AssertionError:
            return True
    return False


def _touching_links(s1, e1, s2, e2):
    return s1 <= e2 and s2 <= e1


def _strength_by_amp(r):
    return (float(r["amp"]), -int(r["window_ap"]), -int(r["t_start"]))


def _strength_latest(r):
    return (float(r["snr"]), int(r["window_ap"]), int(r["t_start"]))


def _count_windows(cands, min_windows=2):
    # windows counted instead of distinct window lengths
    out = pm.baseline_pulses(cands, 1)
    return [p for p in out if p["n_windows"] >= min_windows]


def _count_pulses(cands, min_windows=2, min_baselines=5):
    # baseline pulses counted instead of distinct baselines
    bps = pm.baseline_pulses(cands, min_windows)
    rows = pm.single_pulses(cands, min_windows, 1)
    keep = []
    for pid in sorted({r["pulse"] for r in rows}):
        grp = [r for r in rows if r["pulse"] == pid]
        anchor = max(grp, key=lambda r: (r["snr"], -r["window_ap"], -r["t_start"], -r["baseline"]))
        n = sum(1 for p in bps if p["scan"] == anchor["scan"] and
                p["t_lo"] < anchor["t_hi"] and anchor["t_lo"] < p["t_hi"])
        if n >= min_baselines:
            keep += grp
    return keep


def _transitive_groups(items, strength, span):
    # connected components of the overlap graph instead of anchored groups
    n = len(items)
    seen, groups = [False] * n, []
    for i in range(n):
        if seen[i]:
            continue
        seen[i], comp, stack = True, [i], [i]
        while stack:
            k = stack.pop()
            for j in range(n):
                if not seen[j] and pm._spans_share_ap(*span(items[k]), *span(items[j])):
                    seen[j] = True
                    comp.append(j)
                    stack.append(j)
        groups.append((max(comp, key=lambda k: strength(items[k])), comp))
    return groups


def _loo_keeps_all(tau, dtau_dra, dtau_ddec):
    sol, rms, loo, loo_rms = pm.localize(tau, dtau_dra, dtau_ddec)
    return sol, rms, np.tile(sol, (len(loo), 1)), np.full(len(loo_rms), rms)


def _localize_swapped(tau, dtau_dra, dtau_ddec):
    return pm.localize(tau, dtau_ddec, dtau_dra)


@pytest.mark.parametrize("overrides", [
    dict(_spans_share_ap=_touching_links),
    dict(_window_strength=_strength_by_amp),
    dict(_window_strength=_strength_latest),
    dict(_anchored_groups=_transitive_groups),
    dict(baseline_pulses=_count_windows),
    dict(single_pulses=_count_pulses),
    dict(localize=_loo_keeps_all),
    dict(localize=_localize_swapped),
], ids=["touching-spans", "rep-by-amp", "rep-tie-latest", "transitive-groups", "count-windows",
        "count-pulses", "loo-keeps-all", "partials-swapped"])
def test_planted_mistake_is_caught(overrides):
    assert _fails(_mutant(**overrides))


def test_unmutated_reference_passes_all_checks():
    assert not _fails(pm)




def _partials_hour_angle_flipped(b_xyz, gast, ra, dec):
    return pm.delay_partials(b_xyz, -gast, -ra, dec)


def _partials_no_sign(b_xyz, gast, ra, dec):
    da, dd = pm.delay_partials(b_xyz, gast, ra, dec)
    return -da, -dd


@pytest.mark.parametrize("overrides", [
    dict(delay_partials=_partials_hour_angle_flipped),
    dict(delay_partials=_partials_no_sign),
], ids=["hour-angle-flipped", "partials-sign"])
def test_planted_partials_mistake_is_caught(overrides):
    assert _fails(_mutant(**overrides))
