"""Calibration gains (fringe_set_gains) on cuda:0 against the CPU reference,
which multiplies every sample of baseline b, channel f by g[b][f] before the
search.  Covered: the fused path, the two-pass path (W = 128), the delay-only
search, streaming, an instrumental delay removed exactly, flagged channels,
and NULL gains returning the uncalibrated results bit for bit.
"""

import math

import numpy as np
import pytest

import synth
from fringe_testlib import compare_candidates, compare_windows, oracle_table, run_gpu, to_device

pytestmark = pytest.mark.gpu


def _flat(v):
    return v.reshape(v.shape[0], v.shape[1], -1)


def _gains(rng, nb, f, flag=True):
    g = (rng.uniform(0.5, 1.5, (nb, f)) * np.exp(2j * np.pi * rng.random((nb, f)))).astype(np.complex64)
    if flag:
        g[:, 3:9] = 0
    return g


@pytest.mark.parametrize("case", [
    # (n_bl, T, n_if, n_chan, windows, pad_f, pad_t, flags)
    (3, 400, 8, 32, [1, 2, 4, 8, 16, 32], 4, 2, "batch"),
    (2, 300, 8, 8, [1, 128], 4, 2, "batch"),           # two-pass path
    (2, 500, 4, 16, [1, 2, 4, 8, 16, 32, 64], 2, 2, "delay-only"),
    (2, 260, 16, 64, [2, 8, 32], 4, 2, "batch"),        # F = 1024: 16 folds
], ids=["fused", "two-pass", "delay-only", "wide-band"])
def test_gains_parity(case):
    import paper_2108_05602_amd as F
    nb, t, n_if, n_chan, ws, pf, pt, kind = case
    print(f"case: gains {case}", flush=True)
    rng = np.random.default_rng([55, nb, t, n_if, n_chan])
    v = (rng.standard_normal((nb, t, n_if, n_chan)) +
         1j * rng.standard_normal((nb, t, n_if, n_chan))).astype(np.complex64)
    f = np.arange(n_if * n_chan)
    v[0, t // 3:t // 3 + 6] += (0.9 * np.exp(2j * np.pi * 0.21 * f)).reshape(n_if, n_chan).astype(np.complex64)
    g = _gains(rng, nb, n_if * n_chan)
    d = dict(n_baselines=nb, n_ap=t, n_if=n_if, n_chan=n_chan, ap_seconds=1e-3, chan_width_hz=1e6)
    flags = F.FRINGE_DELAY_ONLY if kind == "delay-only" else 0
    plan, table, cands = run_gpu([d], [v], ws, pf, pt, 4.0, flags=flags, gains=[g])
    ref = oracle_table([v], [d], ws, pf, pt, 4.0, delay_only=(kind == "delay-only"), gains=[g])
    fv = _flat(v) * g[:, None, :]
    n_amb = compare_windows(table, ref, lambda s, b: fv[b], pf, pt, str(case))
    compare_candidates(cands, ref, 4.0, str(case))
    assert n_amb <= max(2, len(ref) // 1000)
    plan.close()


def test_instrumental_delay_removed():
    """A fringe shifted by an instrumental delay of 9 delay bins: with the
    gains that remove it the peak returns to its true bin, amp = W F and
    SNR = sqrt(W F); without them it sits at the shifted bin."""
    print("case: instrumental delay", flush=True)
    w, f, pf, pt, b_true, b_inst, a_rate = 8, 256, 4, 2, 21, 9, 3
    mt, mf = pt * w, pf * f
    t = 64
    u = (np.arange(t) % w)[:, None]
    ff = np.arange(f)[None, :]
    x = np.exp(2j * np.pi * (a_rate * u / mt + (b_true + b_inst) * ff / mf)).astype(np.complex64)
    v = x.reshape(1, t, 8, 32)
    g = np.exp(-2j * np.pi * b_inst * np.arange(f) / mf).astype(np.complex64)[None, :]
    d = dict(n_baselines=1, n_ap=t, n_if=8, n_chan=32, ap_seconds=1.0, chan_width_hz=1.0)
    _, raw, _ = run_gpu([d], [v], [w], pf, pt, 3.0)
    _, cal, _ = run_gpu([d], [v], [w], pf, pt, 3.0, gains=[g])
    aligned = cal[cal["t_start"] % w == 0]
    assert np.all(aligned["k_delay"] == b_true) and np.all(aligned["k_rate"] == a_rate)
    assert np.allclose(aligned["amp"], w * f, rtol=1e-5)
    assert np.allclose(aligned["snr"], math.sqrt(w * f), rtol=1e-5)
    assert np.all(raw[raw["t_start"] % w == 0]["k_delay"] == b_true + b_inst)


def test_null_gains_and_streaming():
    """NULL gains give the never-calibrated records bit for bit; a streamed
    subarray with gains gives the batch search with gains, window for window."""
    import torch

    import paper_2108_05602_amd as F
    print("case: null gains, streamed gains", flush=True)
    spec = synth.evn_scan(5101, 3, 976, 8, 32, 1.024e-3, 16e6, 2, width_max=16, n_tones=1)
    vis = spec.full()
    desc = spec.desc()
    ws = [1, 2, 4, 8, 16, 32]
    rng = np.random.default_rng(7)
    g = _gains(rng, spec.n_baselines, spec.n_freq)
    gd = to_device(g)
    dev = to_device(vis)
    st = torch.cuda.current_stream().cuda_stream
    fields = ("k_rate", "k_delay", "amp", "snr", "energy")
    with F.Plan([desc], ws, snr_threshold=4.5) as p:
        p.search([dev.data_ptr()], st)
        plain = p.windows(np.arange(p.info()["n_windows"]))
        p.set_gains(0, gd.data_ptr())
        p.search([dev.data_ptr()], st)
        calb = p.windows(np.arange(p.info()["n_windows"]))
        p.set_gains(0, None)
        p.search([dev.data_ptr()], st)
        back = p.windows(np.arange(p.info()["n_windows"]))
    for k in fields:
        assert np.array_equal(plain[k], back[k]), k
    assert not np.array_equal(plain["energy"], calb["energy"])
    bmap = {(int(r["baseline"]), int(r["window_ap"]), int(r["t_start"])): r for r in calb}
    chunk = 244
    rows = []
    with F.Plan([dict(desc, n_ap=chunk)], ws, snr_threshold=4.5, flags=F.FRINGE_STREAMING) as p:
        p.set_gains(0, gd.data_ptr())
        for t0 in range(0, vis.shape[1], chunk):
            piece = dev[:, t0:t0 + chunk].contiguous()
            p.search([piece.data_ptr()], st)
            n = p.info()["n_windows"]
            if n:
                rows.append(p.windows(np.arange(n)))
            torch.cuda.synchronize()
    rows = np.concatenate(rows)
    assert len(rows) == len(calb)
    for r in rows:
        b = bmap[(int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))]
        for k in fields:
            assert r[k] == b[k], k


def test_evn_full_scan_with_gains():
    """The full EVN-like scan searched with per-baseline, per-channel gains
    (instrumental delays per IF, phases, amplitude scales, 6 flagged
    channels: the benchmark's calibrated leg), checked against the reference
    on the calibrated data: 300 random windows, the threshold band, 300 windows
    above it, and the candidates."""
    import os

    import torch

    import oracle.fringe_oracle as fo
    import paper_2108_05602_amd as F
    spec = synth.c2()
    p = synth.C2_PARAMS
    print("case: full EVN-like scan with gains", flush=True)
    v = spec.full(threads=min(16, os.cpu_count() or 1))
    fv = v.reshape(spec.n_baselines, spec.n_ap, -1)
    desc = spec.desc()
    rng = np.random.default_rng(7)
    f = np.arange(spec.n_freq)
    tau = np.repeat(rng.uniform(-20e-9, 20e-9, (spec.n_baselines, desc["n_if"])), desc["n_chan"], 1)
    phi = np.repeat(rng.uniform(0, 2 * np.pi, (spec.n_baselines, desc["n_if"])), desc["n_chan"], 1)
    g = (rng.uniform(0.8, 1.2, (spec.n_baselines, spec.n_freq)) *
         np.exp(-1j * (2 * np.pi * f[None, :] * desc["chan_width_hz"] * tau + phi))).astype(np.complex64)
    g[:, 100:106] = 0
    dev = torch.from_numpy(v).to("cuda:0")
    dg = to_device(g)
    stream = torch.cuda.current_stream().cuda_stream
    thr, pf, pt = p["snr_threshold"], p["pad_freq"], p["pad_time"]

    def ref_rows(rows):
        out = []
        m_f = pf * spec.n_freq
        for r_ in rows:
            w, t0, b = int(r_["window_ap"]), int(r_["t_start"]), int(r_["baseline"])
            seg = fo.calibrate(fv[b][None, t0:t0 + w], g[b][None])[0]
            r = fo.search_window(seg, 0, w, pf, pt)
            m_t = pt * w
            out.append((0, b, w, t0, r.k_rate, r.k_delay, r.amp, r.snr, r.energy,
                        fo.signed_bin(r.k_delay, m_f) / (m_f * spec.chan_width_hz),
                        fo.signed_bin(r.k_rate, m_t) / (m_t * spec.ap_seconds), r.margin))
        return np.array(out, dtype=fo.TABLE_DTYPE)

    def run(threshold):
        plan = F.Plan([desc], p["window_aps"], pad_freq=pf, pad_time=pt, snr_threshold=threshold,
                      max_candidates=1 << 20)
        plan.set_gains(0, dg.data_ptr())
        plan.search([dev.data_ptr()], stream)
        return plan

    plan = run(thr)
    cands = plan.candidates()
    rng2 = np.random.default_rng(701)
    srows = plan.windows(np.sort(rng2.choice(plan.info()["n_windows"], 300, replace=False)))
    plan.close()
    low = run(0.99 * thr)
    above = low.candidates()
    low.close()
    band = above[above["snr"] <= 1.01 * thr]
    high = above[above["snr"] > 1.01 * thr]
    print(f"{len(cands)} candidates, {len(band)} in the 1 % band", flush=True)
    assert len(band) < 8000

    def calibrated(s, b):   # only for the rare ambiguous windows
        return fo.calibrate(fv[b][None], g[b][None])[0]

    compare_windows(srows, ref_rows(srows), calibrated, pf, pt, "sample")
    ref_b = ref_rows(band)
    compare_windows(band, ref_b, calibrated, pf, pt, "band")
    pick = np.sort(rng2.choice(len(high), min(300, len(high)), replace=False))
    ref_h = ref_rows(high[pick])
    compare_windows(high[pick], ref_h, calibrated, pf, pt, "high")
    assert np.all(ref_h["snr"] > thr)

    def key(r):
        return (int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))
    got = [key(c) for c in cands]
    assert got == sorted(got)
    want = {key(r) for r in ref_b if r["snr"] > thr} | {key(r) for r in high}
    amb = {key(r) for r in ref_b if abs(r["snr"] - thr) < 1e-4 * thr}
    assert (set(got) ^ want) <= amb
    del dev
