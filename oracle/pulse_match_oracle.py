"""Reference single-pulse matching and delay-only localization, plain Python.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports or runs it;
the test suite does.  Brute force by design (every pair of windows compared,
connected components by breadth-first search, least squares by numpy), so
that it can be checked against the paper by eye.

What is computed (paper, section "Detection rate" criteria and section
"Localization", Eq. (2) with the leave-one-baseline-out check):

  baseline pulses: on one baseline of one scan, candidate windows whose AP
    spans [t_start, t_start + W) share an AP are linked, transitively; a
    linked group is a pulse of that baseline when its windows come from at
    least `min_windows` distinct window lengths.  Its span is the union of
    the spans; its representative is the window of highest SNR (ties: the
    shorter window, then the earlier start).
  single pulses: baseline pulses of one scan whose spans share an AP are
    linked, transitively; a group is a single pulse when it holds at least
    `min_baselines` distinct baselines.  A baseline with several pulses in
    the group is represented by its highest-SNR one.
  localization: over a pulse's baselines, least squares for (dra, ddec) in
    tau_b - tau_cal_b = (dtau/dra)_b dra + (dtau/ddec)_b ddec, and the same
    solve leaving out each baseline in turn.
"""

from __future__ import annotations

from collections import deque

import numpy as np

PULSE_FIELDS = ("scan", "pulse", "baseline", "window_ap", "t_start", "k_rate", "k_delay",
                "amp", "snr", "t_lo", "t_hi", "n_windows", "n_lengths", "delay_s", "rate_hz")


def _spans_share_ap(s1, e1, s2, e2):
    return s1 < e2 and s2 < e1


def _components(n, linked):
    """Connected components of the graph on 0..n-1 with edges linked(i, j)."""
    seen = [False] * n
    comps = []
    for i in range(n):
        if seen[i]:
            continue
        seen[i] = True
        comp, q = [], deque([i])
        while q:
            k = q.popleft()
            comp.append(k)
            for j in range(n):
                if not seen[j] and linked(k, j):
                    seen[j] = True
                    q.append(j)
        comps.append(sorted(comp))
    return comps


def _best(rows, idx):
    return max(idx, key=lambda k: (float(rows[k]["snr"]), -int(rows[k]["window_ap"]),
                                   -int(rows[k]["t_start"])))


def baseline_pulses(cands, min_windows=2):
    """List of dicts (scan, baseline, t_lo, t_hi, n_windows, n_lengths, rep)
    where rep is the representative candidate record."""
    out = []
    keys = sorted({(int(c["scan"]), int(c["baseline"])) for c in cands})
    for scan, b in keys:
        rows = cands[(cands["scan"] == scan) & (cands["baseline"] == b)]
        st = [int(r["t_start"]) for r in rows]
        en = [int(r["t_start"]) + int(r["window_ap"]) for r in rows]
        comps = _components(len(rows), lambda i, j: _spans_share_ap(st[i], en[i], st[j], en[j]))
        for comp in comps:
            lengths = {int(rows[k]["window_ap"]) for k in comp}
            if len(lengths) < min_windows:
                continue
            out.append(dict(scan=scan, baseline=b, t_lo=min(st[k] for k in comp),
                            t_hi=max(en[k] for k in comp), n_windows=len(comp),
                            n_lengths=len(lengths), rep=rows[_best(rows, comp)]))
    return out


def single_pulses(cands, min_windows=2, min_baselines=5):
    """Rows (one per single pulse and baseline) as a list of dicts with the
    PULSE_FIELDS, in (scan, pulse start, baseline) order; pulses numbered
    from 0 in that order over all scans."""
    bps = baseline_pulses(cands, min_windows)
    rows = []
    groups = []
    for scan in sorted({p["scan"] for p in bps}):
        ps = [p for p in bps if p["scan"] == scan]
        comps = _components(len(ps), lambda i, j: _spans_share_ap(ps[i]["t_lo"], ps[i]["t_hi"],
                                                                  ps[j]["t_lo"], ps[j]["t_hi"]))
        for comp in comps:
            if len({ps[k]["baseline"] for k in comp}) < min_baselines:
                continue
            groups.append((scan, min(ps[k]["t_lo"] for k in comp), [ps[k] for k in comp]))
    groups.sort(key=lambda g: (g[0], g[1]))
    for pid, (scan, _, members) in enumerate(groups):
        by_b = {}
        for p in members:
            q = by_b.get(p["baseline"])
            if q is None or (float(p["rep"]["snr"]), -p["t_lo"]) > (float(q["rep"]["snr"]), -q["t_lo"]):
                by_b[p["baseline"]] = p
        for b in sorted(by_b):
            p = by_b[b]
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
