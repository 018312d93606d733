"""The autotuner (FRINGE_AUTOTUNE) on cuda:0.

A plan of uneven scans (bands of 256 and 1,024 channels, windows 1-64 APs)
made with the flag tunes each class of its scans once (search mode x time
chunk, timed on a synthetic sample) and records the choice in the tune
table.  Its records equal the default plan's bit for bit wherever the tuned
mode is the default one (the chunk never changes a result), and otherwise
agree with the CPU reference; a second tuned plan reuses the table without
tuning again; the table survives a save / clear / load round trip."""

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import synth
from fringe_testlib import compare_windows, run_gpu

pytestmark = pytest.mark.gpu

FIELDS = ("scan", "baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy")


def test_autotuned_plans(tmp_path):
    import paper_2108_05602_amd as F
    print("case: autotuned plan of uneven scans", flush=True)
    specs = [synth.evn_scan(5100, 4, 700, 8, 32, 1.024e-3, 16e6, 2, width_max=16, n_tones=1),
             synth.evn_scan(5101, 3, 600, 16, 64, 1.024e-3, 16e6, 2, width_max=16),
             synth.evn_scan(5102, 5, 450, 8, 32, 1.024e-3, 16e6, 1, width_max=8)]
    vis = [s.full() for s in specs]
    descs = [s.desc() for s in specs]
    ws, pf, pt, thr = [1, 2, 4, 8, 16, 32, 64], 4, 2, 4.5
    F.fringe_tune_clear()
    tuned, t_tab, t_c = run_gpu(descs, vis, ws, pf, pt, thr, flags=F.FRINGE_AUTOTUNE)
    entries = tuned.tuning()
    print("tune entries:", entries, flush=True)
    assert sorted(e["n_freq"] for e in entries) == [256, 1024]
    for e in entries:
        assert e["spectra"] in (0, 1) and e["chunk"] in (128, 256, 512, 1024)
        assert e["pad_freq"] == pf and e["pad_time"] == pt and e["log2_wmax"] == 6
        assert e["ms_fused"] > 0
        best = min(m for m in (e["ms_fused"], e["ms_spectra"]) if m > 0)
        assert (e["ms_spectra"] if e["spectra"] else e["ms_fused"]) == best
    default, d_tab, d_c = run_gpu(descs, vis, ws, pf, pt, thr)
    by_f = {e["n_freq"]: e for e in entries}
    for s, sp in enumerate(specs):
        tsub, dsub = t_tab[t_tab["scan"] == s], d_tab[d_tab["scan"] == s]
        default_spectra = 1 if sp.n_freq >= 1024 else 0
        if by_f[sp.n_freq]["spectra"] == default_spectra:
            for k in FIELDS:
                assert np.array_equal(tsub[k], dsub[k]), (s, k)
        else:
            ref, _ = fo.search_scan(vis[s], ws, pf, pt, thr, sp.ap_seconds, sp.chan_width_hz,
                                    scan=s)
            fv = vis[s].reshape(sp.n_baselines, sp.n_ap, -1)
            compare_windows(tsub, ref, lambda sc, b: fv[b], pf, pt, f"tuned scan {s}")
    # a second tuned plan takes the table's entries as they are
    again, _, _ = run_gpu(descs[:2], vis[:2], ws, pf, pt, thr, flags=F.FRINGE_AUTOTUNE,
                          all_windows=False)
    assert sorted(again.tuning(), key=lambda e: e["n_freq"]) == \
        sorted(entries, key=lambda e: e["n_freq"])
    path = str(tmp_path / "tune.json")
    F.fringe_tune_save(path)
    F.fringe_tune_clear()
    F.fringe_tune_load(path)
    third, _, _ = run_gpu(descs[1:2], vis[1:2], ws, pf, pt, thr, flags=F.FRINGE_AUTOTUNE,
                          all_windows=False)
    assert third.tuning() == [by_f[1024]]
    for p in (tuned, default, again, third):
        p.close()
