"""Reference single-pulse matching and delay-only localization, plain Python.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports or runs it;
the test suite does.  Brute force by design (each anchor compared with every
remaining item, distinct counts by sets, least squares by numpy), so that it
can be checked against the paper by eye.

What is computed (paper: the single-pulse criteria of section "Detection
rate"; Eq. (2) of section "Localization"; the leave-one-baseline-out check
of section "Localization accuracy").  The criteria name no grouping rule; groups
here are anchored at their strongest member, so that a long-lived RFI
signal cannot chain distinct pulses into one:

  baseline pulses: on one baseline of one scan, repeatedly take the
    strongest remaining candidate window (highest SNR; ties: the shorter
    window, then the earlier start) and every remaining window whose AP
    span [t_start, t_start + W) shares an AP with it; remove them.  The
    group is a pulse of that baseline when its windows come from at least
    `min_windows` distinct window lengths.  Its span is the union of its
    windows' spans, its representative the anchor window.
  single pulses: among the baseline pulses of one scan, repeatedly take the
    strongest remaining one (by its representative: SNR, then the shorter
    window, the earlier start, the lower baseline) and every remaining one
    whose span shares an AP with its span; remove them.  The group is a
    single pulse when it holds at least `min_baselines` distinct baselines;
    a baseline with several pulses in it is represented by its strongest.
    Single pulses are numbered from 0 over all scans in (scan, first AP of
    the group, order found) order, rows within a pulse by baseline.
  localization: over a pulse's baselines, least squares for (dra, ddec) in
    tau_b - tau_cal_b = (dtau/dra)_b dra + (dtau/ddec)_b ddec, and the same
    solve leaving out each baseline in turn.
  partials: of the geometric delay tau_g = t_2 - t_1 = -(b . s) / c of a
    baseline b = r_2 - r_1 (Earth-fixed metres) toward a source at (ra, dec)
    whose Greenwich hour angle is gast - ra (no precession, nutation, polar
    motion or aberration: the a priori geometry of a small offset solve).
"""

from __future__ import annotations

import numpy as np

PULSE_FIELDS = ("scan", "pulse", "baseline", "window_ap", "t_start", "k_rate", "k_delay",
                "amp", "snr", "t_lo", "t_hi", "n_windows", "n_lengths", "delay_s", "rate_hz")


def _spans_share_ap(s1, e1, s2, e2):
    return s1 < e2 and s2 < e1


def _window_strength(r):
    return (float(r["snr"]), -int(r["window_ap"]), -int(r["t_start"]))


def _anchored_groups(items, strength, span):
    """Groups of `items`: repeatedly the strongest remaining item and every
    remaining item whose span shares an AP with the anchor's; returns
    (anchor, members) pairs in the order found."""
    left = list(range(len(items)))
    groups = []
    while left:
        anchor = max(left, key=lambda k: strength(items[k]))
        s0, e0 = span(items[anchor])
        members = [k for k in left if _spans_share_ap(*span(items[k]), s0, e0)]
        left = [k for k in left if k not in members]
        groups.append((anchor, members))
    return groups


def baseline_pulses(cands, min_windows=2):
    """List of dicts (scan, baseline, t_lo, t_hi, n_windows, n_lengths, rep)
    where rep is the representative candidate record."""
    out = []
    keys = sorted({(int(c["scan"]), int(c["baseline"])) for c in cands})
    for scan, b in keys:
        rows = cands[(cands["scan"] == scan) & (cands["baseline"] == b)]
        span = lambda r: (int(r["t_start"]), int(r["t_start"]) + int(r["window_ap"]))
        for anchor, members in _anchored_groups(rows, _window_strength, span):
            lengths = {int(rows[k]["window_ap"]) for k in members}
            if len(lengths) < min_windows:
                continue
            out.append(dict(scan=scan, baseline=b, t_lo=min(span(rows[k])[0] for k in members),
                            t_hi=max(span(rows[k])[1] for k in members),
                            n_windows=len(members), n_lengths=len(lengths), rep=rows[anchor]))
    return out


def _pulse_strength(p):
    return _window_strength(p["rep"]) + (-p["baseline"],)


def single_pulses(cands, min_windows=2, min_baselines=5):
    """Rows (one per single pulse and baseline) as a list of dicts with the
    PULSE_FIELDS, in (pulse, baseline) order."""
    bps = baseline_pulses(cands, min_windows)
    found = []
    for scan in sorted({p["scan"] for p in bps}):
        ps = [p for p in bps if p["scan"] == scan]
        groups = _anchored_groups(ps, _pulse_strength, lambda p: (p["t_lo"], p["t_hi"]))
        for order, (_, members) in enumerate(groups):
            if len({ps[k]["baseline"] for k in members}) < min_baselines:
                continue
            found.append((scan, min(ps[k]["t_lo"] for k in members), order,
                          [ps[k] for k in members]))
    found.sort(key=lambda g: g[:3])
    rows = []
    for pid, (scan, _, _, members) in enumerate(found):
        for b in sorted({p["baseline"] for p in members}):
            p = max((q for q in members if q["baseline"] == b), key=_pulse_strength)
            r = p["rep"]
            rows.append(dict(scan=scan, pulse=pid, baseline=b, window_ap=int(r["window_ap"]),
                             t_start=int(r["t_start"]), k_rate=int(r["k_rate"]),
                             k_delay=int(r["k_delay"]), amp=float(r["amp"]), snr=float(r["snr"]),
                             t_lo=p["t_lo"], t_hi=p["t_hi"], n_windows=p["n_windows"],
                             n_lengths=p["n_lengths"], delay_s=float(r["delay_s"]),
                             rate_hz=float(r["rate_hz"])))
    return rows


def localize(tau, dtau_dra, dtau_ddec):
    """Least-squares (dra, ddec) of Eq. (2) from residual delays tau (already
    minus the fine-calibration delays) and the partials per baseline, with
    the RMS of its delay residuals; and, for three or more baselines, the
    solution and residual RMS (over the kept baselines) leaving out each one.
    Returns (sol (2,), rms, loo (n, 2), loo_rms (n,))."""
    a = np.column_stack([np.asarray(dtau_dra, float), np.asarray(dtau_ddec, float)])
    y = np.asarray(tau, float)

    def fit(aa, yy):
        x = np.linalg.lstsq(aa, yy, rcond=None)[0]
        return x, float(np.sqrt(np.mean((yy - aa @ x) ** 2)))

    sol, rms = fit(a, y)
    loo, loo_rms = [], []
    if len(y) >= 3:
        for i in range(len(y)):
            keep = np.arange(len(y)) != i
            x, r = fit(a[keep], y[keep])
            loo.append(x)
            loo_rms.append(r)
    return sol, rms, np.array(loo).reshape(-1, 2), np.array(loo_rms)


C_LIGHT = 299792458.0


def delay_partials(b_xyz, gast, ra, dec):
    """(dtau/dra, dtau/ddec) in s/rad for each Earth-fixed baseline vector
    b_xyz[i] = r_2 - r_1 (metres).  The source direction in the Earth-fixed
    frame is s = (cos dec cos h, -cos dec sin h, sin dec) with h = gast - ra,
    and tau_g = -(b . s) / c; the partials differentiate s."""
    b = np.asarray(b_xyz, float).reshape(-1, 3)
    h = gast - ra
    ds_dra = np.array([np.cos(dec) * np.sin(h), np.cos(dec) * np.cos(h), 0.0])
    ds_ddec = np.array([-np.sin(dec) * np.cos(h), np.sin(dec) * np.sin(h), np.cos(dec)])
    return -(b @ ds_dra) / C_LIGHT, -(b @ ds_ddec) / C_LIGHT
