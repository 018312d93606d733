"""The candidate consumers on the output of the GPU search.

  * A small EVN-like scan with two whole-scan RFI tones: the GPU search plus
    fringe_match against the reference search plus the reference matching.
    Windows whose SNRs lie within the 1e-4 bar of one another may swap as
    group anchors, so what is compared is what such a swap cannot move: the
    number of single pulses, a one-to-one pairing of them by time, and for
    every detection with SNR >= 6 on either side, the same baseline in the
    paired pulse with its SNR within 1e-4.
  * The full EVN-like scan (20 pulses, 10 RFI tones): every injected pulse is
    found as exactly one single pulse, and every single pulse covers an
    injected one.
"""

import os

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import oracle.pulse_match_oracle as pm
import synth
from fringe_testlib import run_gpu

pytestmark = pytest.mark.gpu

W = [1, 2, 4, 8, 16, 32]


def _groups(rows, pulse_key):
    out = {}
    for r in rows:
        out.setdefault(int(r[pulse_key]), []).append(r)
    return out


def _span(rows):
    return min(int(r["t_lo"]) for r in rows), max(int(r["t_hi"]) for r in rows)


def test_match_after_gpu_search():
    import paper_2108_05602_amd as F
    spec = synth.c2(seed=21, n_stations=6, n_ap=1500, n_pulses=4, n_tones=2)
    print("case: match, 6 stations x 1500 AP, seed 21", flush=True)
    vis = spec.full(threads=4)
    _, _, cands = run_gpu([spec.desc()], [vis], W, 4, 2, 4.5, all_windows=False)
    got, n_got = F.fringe_match(cands, 2, 5)
    _, ref_c = fo.search_scan(vis, W, 4, 2, 4.5, spec.ap_seconds, spec.chan_width_hz)
    ref = pm.single_pulses(ref_c, 2, 5)
    g_by, r_by = _groups(got, "pulse"), _groups(ref, "pulse")
    assert n_got == len(r_by) == 4
    pair = {}
    for pid, rows in r_by.items():
        lo, hi = _span(rows)
        hits = [q for q, g in g_by.items() if _span(g)[0] < hi and lo < _span(g)[1]]
        assert len(hits) == 1, (pid, lo, hi, hits)
        pair[pid] = hits[0]
    assert sorted(pair.values()) == sorted(g_by)
    for pid, q in pair.items():
        g_snr = {int(r["baseline"]): float(r["snr"]) for r in g_by[q]}
        r_snr = {int(r["baseline"]): float(r["snr"]) for r in r_by[pid]}
        for b in set(g_snr) | set(r_snr):
            if max(g_snr.get(b, 0.0), r_snr.get(b, 0.0)) < 6.0:
                continue
            assert b in g_snr and b in r_snr, (pid, b)
            assert abs(g_snr[b] - r_snr[b]) <= 1e-4 * r_snr[b], (pid, b, g_snr[b], r_snr[b])


def test_match_full_scan_recovers_injected_pulses():
    import torch

    import paper_2108_05602_amd as F
    spec = synth.c2()
    p = synth.C2_PARAMS
    print("case: match, full EVN-like scan", flush=True)
    v = spec.full(threads=min(16, os.cpu_count() or 1))
    dev = torch.from_numpy(v).to("cuda:0")
    del v
    with F.Plan([spec.desc()], p["window_aps"], pad_freq=p["pad_freq"], pad_time=p["pad_time"],
                snr_threshold=p["snr_threshold"], max_candidates=1 << 20) as plan:
        plan.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        cands = plan.candidates()
    rows, n_p = F.fringe_match(cands, 2, 5)
    spans = {pid: _span(g) for pid, g in _groups(rows, "pulse").items()}
    for q in spec.pulses:
        hits = [pid for pid, (lo, hi) in spans.items() if lo < q.start + q.width and q.start < hi]
        assert len(hits) == 1, (q.start, q.width, q.snr, hits)
    for pid, (lo, hi) in spans.items():
        assert any(lo < q.start + q.width and q.start < hi for q in spec.pulses), (pid, lo, hi)
    assert n_p == len(spec.pulses)
