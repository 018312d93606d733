"""The large dense scan at full size (66 baselines x 117200 APs x 1024
channels of 0.512 ms APs, 63.4 GB; windows 1-128 APs, 23.1 M windows): the
two-pass path (delay transform to HBM, then rate transform and peak) on
cuda:0, checked against the CPU reference on samples: 150 random windows,
150 windows drawn from those within 1 % of the threshold (found by a second
search at 0.99 x threshold), 100 from above that band; and properties of the
whole candidate list (ordered, its records equal to the low-threshold
search's, every window of the low search above 1.01 x threshold in it and
none below 0.99 x)."""

import os

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import synth
from fringe_testlib import compare_windows

pytestmark = pytest.mark.gpu


def test_large_dense_scan_full_size():
    import torch

    import paper_2108_05602_amd as F
    spec = synth.c5()
    p = synth.C5_PARAMS
    print(f"case: large dense scan {spec.n_baselines} BL x {spec.n_ap} AP x {spec.n_freq} ch "
          f"({spec.nbytes() / 1e9:.1f} GB)", flush=True)
    v = spec.full(threads=min(16, os.cpu_count() or 1))
    fv = v.reshape(spec.n_baselines, spec.n_ap, -1)
    dev = torch.from_numpy(v).to("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    thr, pf, pt = p["snr_threshold"], p["pad_freq"], p["pad_time"]
    common = dict(pad_freq=pf, pad_time=pt, max_candidates=1 << 22)
    rng = np.random.default_rng(55)
    with F.Plan([spec.desc()], p["window_aps"], snr_threshold=thr, flags=F.FRINGE_PROFILE,
                **common) as plan:
        for _ in range(2):   # the second search is the one reported (warm)
            plan.search([dev.data_ptr()], stream)
            cands = plan.candidates()
        prof = plan.profile()
        n_win = plan.info()["n_windows"]
        ms = prof["delay_ms"] + prof["rate_ms"] + prof["finalize_ms"] + prof["compact_ms"]
        print(f"kernels {prof}: {n_win / (ms * 1e-3) / 1e6:.1f} M windows/s", flush=True)
        assert n_win == 23084226
        srows = plan.windows(np.sort(rng.choice(n_win, 150, replace=False)))
    print(f"{len(cands)} candidates", flush=True)
    with F.Plan([spec.desc()], p["window_aps"], snr_threshold=0.99 * thr, **common) as low:
        low.search([dev.data_ptr()], stream)
        above = low.candidates()
    band = above[above["snr"] <= 1.01 * thr]
    high = above[above["snr"] > 1.01 * thr]
    print(f"{len(above)} above 0.99 x threshold, {len(band)} in the 1 % band", flush=True)

    def ref_rows(rows):
        out = []
        m_f = pf * spec.n_freq
        for g in rows:
            w, t0, b = int(g["window_ap"]), int(g["t_start"]), int(g["baseline"])
            r = fo.search_window(fv[b], t0, w, pf, pt)
            m_t = pt * w
            out.append((0, b, w, t0, r.k_rate, r.k_delay, r.amp, r.snr, r.energy,
                        fo.signed_bin(r.k_delay, m_f) / (m_f * spec.chan_width_hz),
                        fo.signed_bin(r.k_rate, m_t) / (m_t * spec.ap_seconds), r.margin))
        return np.array(out, dtype=fo.TABLE_DTYPE)

    compare_windows(srows, ref_rows(srows), lambda s, b: fv[b], pf, pt, "sample")
    pb = band[np.sort(rng.choice(len(band), min(150, len(band)), replace=False))]
    compare_windows(pb, ref_rows(pb), lambda s, b: fv[b], pf, pt, "band")
    ph = high[np.sort(rng.choice(len(high), min(100, len(high)), replace=False))]
    ref_h = ref_rows(ph)
    compare_windows(ph, ref_h, lambda s, b: fv[b], pf, pt, "high")
    assert np.all(ref_h["snr"] > thr)

    def key(r):
        return (int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))
    got = [key(c) for c in cands]
    assert got == sorted(got)
    low_by_key = {key(r): r for r in above}
    for c in cands:
        r = low_by_key[key(c)]
        assert (r["k_rate"], r["k_delay"], r["amp"], r["snr"]) == (c["k_rate"], c["k_delay"], c["amp"], c["snr"])
    assert {key(r) for r in high} <= set(got)
    assert np.all(cands["snr"] > thr)
    del dev
