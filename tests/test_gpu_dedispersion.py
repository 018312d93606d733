"""Dedispersion shifts (fringe_set_shifts) on cuda:0 against the CPU
reference, which moves channel f of every AP t to t - d_f (0 past the data)
before the search.

Covered: the fused path (windows to 32 and to 64 APs), the two-pass path
(W = 128), the delay-only search, shifts with calibration gains, a
dispersed pulse restored exactly, and a batch of DM trials searched as
scans of one plan over one cube (one launch) equal to separate plans.  The
cubes are followed in device memory by NaN samples, so a read past a
baseline's data that was not turned into zeros would show in the results.
"""

import math

import numpy as np
import pytest

import synth
from fringe_testlib import compare_candidates, compare_windows, oracle_table, to_device

pytestmark = pytest.mark.gpu


def _padded(v):
    """The cube on the device followed by NaN samples, T + 64 APs of them (more
    than any read past the last baseline could reach: shifts are clamped to
    T); returns (tensor, ptr)."""
    import torch
    v = np.ascontiguousarray(v)
    t, nf = v.shape[1], int(np.prod(v.shape[2:]))
    flat = torch.from_numpy(v.reshape(-1))
    buf = torch.full((flat.numel() + (t + 64) * nf,), complex(float("nan"), float("nan")),
                     dtype=torch.complex64, device="cuda")
    buf[:flat.numel()].copy_(flat.cuda())
    return buf, buf.data_ptr()


def _run(descs, ptrs, ws, pf, pt, thr, flags=0, shifts=None, gains=None):
    import torch

    import paper_2108_05602_amd as F
    keep = []
    plan = F.Plan(descs, ws, pad_freq=pf, pad_time=pt, snr_threshold=thr, flags=flags,
                  max_candidates=1 << 16)
    for s in range(len(descs)):
        if shifts is not None and shifts[s] is not None:
            keep.append(to_device(np.asarray(shifts[s], dtype=np.int32)))
            plan.set_shifts(s, keep[-1].data_ptr())
        if gains is not None and gains[s] is not None:
            keep.append(to_device(np.asarray(gains[s], dtype=np.complex64)))
            plan.set_gains(s, keep[-1].data_ptr())
    plan.search(ptrs, torch.cuda.current_stream().cuda_stream)
    table = plan.windows(np.arange(plan.info()["n_windows"]))
    cands = plan.candidates()
    torch.cuda.synchronize()
    return plan, table, cands


def _shifted(v, d):
    out = np.zeros_like(v)
    for f, k in enumerate(d):
        if k < v.shape[1]:
            out[:, :v.shape[1] - k, f] = v[:, k:, f]
    return out


@pytest.mark.parametrize("case", [
    # (n_bl, T, n_if, n_chan, windows, pad_f, pad_t, kind, max shift)
    (3, 400, 8, 32, [1, 2, 4, 8, 16, 32], 4, 2, "full", 40),
    (2, 300, 4, 16, [1, 4, 16, 64], 4, 2, "full", 90),
    (2, 300, 8, 8, [1, 128], 4, 2, "full", 35),          # two-pass path
    (2, 500, 4, 16, [1, 2, 4, 8, 16, 32], 2, 2, "delay-only", 60),
    (2, 260, 8, 32, [2, 8, 32], 4, 1, "gains", 300),      # shifts past the data too
], ids=["fused32", "fused64", "two-pass", "delay-only", "with-gains"])
def test_shift_parity(case):
    import paper_2108_05602_amd as F
    nb, t, n_if, n_chan, ws, pf, pt, kind, dmax = case
    print(f"case: shifts {case}", flush=True)
    rng = np.random.default_rng([66, nb, t, n_if, n_chan])
    nf = n_if * n_chan
    v = (rng.standard_normal((nb, t, n_if, n_chan)) +
         1j * rng.standard_normal((nb, t, n_if, n_chan))).astype(np.complex64)
    d = np.sort(rng.integers(0, dmax + 1, nf))[::-1].astype(np.int32)
    fv = v.reshape(nb, t, nf)
    # a dispersed fringe that the shifts bring back together
    f = np.arange(nf)
    for k in range(5):
        rows = t // 3 + k + d
        ok = rows < t
        fv[0, rows[ok], f[ok]] += (0.9 * np.exp(2j * np.pi * 0.19 * f[ok])).astype(np.complex64)
    g = None
    if kind == "gains":
        g = (rng.uniform(0.5, 1.5, (nb, nf)) * np.exp(2j * np.pi * rng.random((nb, nf)))).astype(np.complex64)
    desc = dict(n_baselines=nb, n_ap=t, n_if=n_if, n_chan=n_chan, ap_seconds=1e-3, chan_width_hz=1e6)
    buf, ptr = _padded(v)
    flags = F.FRINGE_DELAY_ONLY if kind == "delay-only" else 0
    plan, table, cands = _run([desc], [ptr], ws, pf, pt, 4.0, flags=flags, shifts=[d],
                              gains=[g] if g is not None else None)
    ref = oracle_table([v], [desc], ws, pf, pt, 4.0, delay_only=(kind == "delay-only"),
                       gains=[g] if g is not None else None, shifts=[d])
    xs = _shifted(fv * (g[:, None, :] if g is not None else 1), d)
    n_amb = compare_windows(table, ref, lambda s, b: xs[b], pf, pt, str(case))
    compare_candidates(cands, ref, 4.0, str(case))
    assert n_amb <= max(2, len(ref) // 1000)
    assert np.all(np.isfinite(table["amp"]))
    plan.close()
    del buf


def test_dispersed_pulse_restored():
    """A unit pulse reaching channel f at AP t0 + d_f: with the shifts the
    one-AP window at t0 has amp = F and SNR = sqrt(F) at delay bin 0."""
    print("case: dispersed pulse", flush=True)
    nf, t, t0 = 256, 200, 17
    d = (np.arange(nf)[::-1] * 150) // nf
    v = np.zeros((1, t, nf), np.complex64)
    v[0, t0 + d, np.arange(nf)] = 1.0
    desc = dict(n_baselines=1, n_ap=t, n_if=8, n_chan=32, ap_seconds=1.0, chan_width_hz=1.0)
    buf, ptr = _padded(v)
    _, table, _ = _run([desc], [ptr], [1], 4, 2, 3.0, shifts=[d.astype(np.int32)])
    r = table[table["t_start"] == t0][0]
    assert (int(r["k_rate"]), int(r["k_delay"])) == (0, 0)
    assert r["amp"] == pytest.approx(nf, rel=1e-6)
    assert r["snr"] == pytest.approx(math.sqrt(nf), rel=1e-6)
    assert np.all(table[table["t_start"] != t0]["amp"] == 0)


def test_dm_trials_one_launch():
    """Four DM trials of one EVN-like slice as four scans of one plan over the
    same device cube: one fused launch, each scan equal to its own plan."""
    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    print("case: DM trials", flush=True)
    spec = synth.evn_scan(5201, 3, 1200, 8, 32, 1.024e-3, 16e6, 2, width_max=16, n_tones=1)
    v = spec.full()
    desc = spec.desc()
    freqs = channel_freqs_hz(1.6e9, 8, 32, desc["chan_width_hz"])
    trials = [dm_shifts(dm, freqs, desc["ap_seconds"]) for dm in (0.0, 40.0, 120.0, 300.0)]
    assert trials[-1].max() > 50
    ws = [1, 2, 4, 8, 16, 32]
    buf, ptr = _padded(v)
    plan, table, cands = _run([desc] * 4, [ptr] * 4, ws, 4, 2, 4.5, flags=F.FRINGE_PROFILE,
                              shifts=trials)
    prof = plan.profile()
    assert prof["rate_launches"] == 1, prof
    for s, d in enumerate(trials):
        _, t1, _ = _run([desc], [ptr], ws, 4, 2, 4.5, shifts=[d])
        sub = table[table["scan"] == s]
        for k in ("baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy"):
            assert np.array_equal(sub[k], t1[k]), (s, k)
    # DM 0 is the unshifted search
    _, t0, _ = _run([desc], [ptr], ws, 4, 2, 4.5)
    for k in ("k_delay", "amp", "snr"):
        assert np.array_equal(table[table["scan"] == 0][k], t0[k]), k
    plan.close()
    del buf


def test_shift_errors():
    import torch

    import paper_2108_05602_amd as F
    print("case: shift errors", flush=True)
    desc = dict(n_baselines=1, n_ap=100, n_if=2, n_chan=32, ap_seconds=1e-3, chan_width_hz=1e6)
    d = torch.zeros(64, dtype=torch.int32, device="cuda")
    v = torch.zeros((1, 100, 2, 32), dtype=torch.complex64, device="cuda")
    # streaming plans take shifts before their first search, not after
    with F.Plan([desc], [4], flags=F.FRINGE_STREAMING) as p:
        p.set_shifts(0, d.data_ptr())
        p.search([v.data_ptr()], torch.cuda.current_stream().cuda_stream)
        with pytest.raises(F.FringeError) as e:
            p.set_shifts(0, d.data_ptr())
        assert e.value.code == -6
    with F.Plan([desc], [4], flags=F.FRINGE_PLAIN) as p:
        with pytest.raises(F.FringeError) as e:
            p.set_shifts(0, d.data_ptr())
        assert e.value.code == -2
        p.set_shifts(0, None)
    with F.Plan([desc], [4]) as p:
        with pytest.raises(F.FringeError) as e:
            p.set_shifts(1, d.data_ptr())
        assert e.value.code == -1


# ------------------------------------------ the dedispersion pass (fringe_dedisperse) ---

def test_dedisperse_pass_matches_reference():
    """The pass moves channel f of AP t + d_f to AP t, zeros past the data,
    clamps the shifts to [0, n_ap]: exactly the reference's dedispersion,
    sample for sample; the input is followed by NaN samples, so a read past
    a baseline's data would show."""
    import torch

    import oracle.fringe_oracle as fo
    import paper_2108_05602_amd as F
    rng = np.random.default_rng(77)
    n_bl, t, nf = 3, 200, 64
    print(f"case: dedisperse pass {n_bl} x {t} x {nf}", flush=True)
    v = (rng.normal(size=(n_bl, t, nf)) + 1j * rng.normal(size=(n_bl, t, nf))).astype(np.complex64)
    d = rng.integers(-5, 260, nf).astype(np.int32)
    d[:3] = [0, t, t + 7]                      # none, all past the data, clamped
    buf, ptr = _padded(v)
    out = torch.full((n_bl * t * nf,), complex(1.0, 1.0), dtype=torch.complex64, device="cuda")
    dd = to_device(d)
    F.fringe_dedisperse(ptr, out.data_ptr(), n_bl, t, nf, dd.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n_bl, t, nf)
    ref = fo.dedisperse(v, np.clip(d, 0, t)).astype(np.complex64)
    assert np.array_equal(got, ref)
    del buf


@pytest.mark.parametrize("delay_only", [False, True], ids=["full", "delay-only"])
def test_dedisperse_pass_then_search_equals_shifted_search(delay_only):
    """Searching the dedispersed cube without shifts gives, bit for bit, what
    the plan's own shifts give on the original cube."""
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    spec = synth.c2(seed=5, n_stations=4, n_ap=700, n_pulses=3, n_tones=1)
    print(f"case: dedisperse pass then search, delay_only={delay_only}", flush=True)
    v = spec.full(threads=4)
    desc = spec.desc()
    freqs = channel_freqs_hz(1.6e9, desc["n_if"], desc["n_chan"], desc["chan_width_hz"])
    d = dm_shifts(300.0, freqs, desc["ap_seconds"])
    ws = [1, 2, 4, 8, 16, 32]
    flags = F.FRINGE_DELAY_ONLY if delay_only else 0
    buf, ptr = _padded(v)
    _, t_shift, c_shift = _run([desc], [ptr], ws, 4, 2, 4.5, flags=flags, shifts=[d])
    out = torch.empty(v.size, dtype=torch.complex64, device="cuda")
    dd = to_device(d.astype(np.int32))
    F.fringe_dedisperse(ptr, out.data_ptr(), spec.n_baselines, spec.n_ap, spec.n_freq,
                        dd.data_ptr(), torch.cuda.current_stream().cuda_stream)
    _, t_pass, c_pass = _run([desc], [out.data_ptr()], ws, 4, 2, 4.5, flags=flags)
    assert t_shift.tobytes() == t_pass.tobytes()
    assert c_shift.tobytes() == c_pass.tobytes()
    del buf


def test_evn_full_scan_one_dm_trial():
    """The full EVN-like scan searched with the shifts of DM 500 (the largest
    trial of the benchmark's DM search, shifts up to 112 APs), checked
    against the reference on the dedispersed data: 300 random windows, every
    window within 1 % of the threshold, 300 above it, and the candidates."""
    import os

    import torch

    import oracle.fringe_oracle as fo
    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    spec = synth.c2()
    p = synth.C2_PARAMS
    print("case: full EVN-like scan, DM 500", flush=True)
    v = spec.full(threads=min(16, os.cpu_count() or 1))
    fv = v.reshape(spec.n_baselines, spec.n_ap, -1)
    desc = spec.desc()
    freqs = channel_freqs_hz(1.6e9, desc["n_if"], desc["n_chan"], desc["chan_width_hz"])
    d = dm_shifts(500.0, freqs, desc["ap_seconds"]).astype(np.int32)
    dmax = int(d.max())
    dev = torch.from_numpy(v).to("cuda:0")
    dd = to_device(d)
    stream = torch.cuda.current_stream().cuda_stream
    thr, pf, pt = p["snr_threshold"], p["pad_freq"], p["pad_time"]
    t_all = spec.n_ap

    def ref_rows(rows):
        out = []
        m_f = pf * spec.n_freq
        for g in rows:
            w, t0, b = int(g["window_ap"]), int(g["t_start"]), int(g["baseline"])
            # the reference's dedispersion of a slice reaching dmax APs past the
            # window (or the scan's end) equals the whole scan's on the window
            sl = fv[b][None, t0:min(t_all, t0 + w + dmax)]
            seg = fo.dedisperse(sl, np.minimum(d, sl.shape[1]))[0, :w]
            r = fo.search_window(seg, 0, w, pf, pt)
            m_t = pt * w
            out.append((0, b, w, t0, r.k_rate, r.k_delay, r.amp, r.snr, r.energy,
                        fo.signed_bin(r.k_delay, m_f) / (m_f * spec.chan_width_hz),
                        fo.signed_bin(r.k_rate, m_t) / (m_t * spec.ap_seconds), r.margin))
        return np.array(out, dtype=fo.TABLE_DTYPE)

    def run(threshold):
        plan = F.Plan([desc], p["window_aps"], pad_freq=pf, pad_time=pt, snr_threshold=threshold,
                      max_candidates=1 << 20)
        plan.set_shifts(0, dd.data_ptr())
        plan.search([dev.data_ptr()], stream)
        return plan

    plan = run(thr)
    cands = plan.candidates()
    rng = np.random.default_rng(500)
    n_win = plan.info()["n_windows"]
    srows = plan.windows(np.sort(rng.choice(n_win, 300, replace=False)))
    plan.close()
    low = run(0.99 * thr)
    above = low.candidates()
    low.close()
    band = above[above["snr"] <= 1.01 * thr]
    high = above[above["snr"] > 1.01 * thr]
    print(f"{len(cands)} candidates, {len(band)} in the 1 % band", flush=True)
    assert len(band) < 8000

    def dedispersed(s, b):   # only for the rare ambiguous windows
        return fo.dedisperse(fv[b][None], d)[0]

    compare_windows(srows, ref_rows(srows), dedispersed, pf, pt, "sample")
    ref_b = ref_rows(band)
    compare_windows(band, ref_b, dedispersed, pf, pt, "band")
    pick = np.sort(rng.choice(len(high), min(300, len(high)), replace=False))
    ref_h = ref_rows(high[pick])
    compare_windows(high[pick], ref_h, dedispersed, pf, pt, "high")
    assert np.all(ref_h["snr"] > thr)

    def key(r):
        return (int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))
    got = [key(c) for c in cands]
    assert got == sorted(got)
    want = {key(r) for r in ref_b if r["snr"] > thr} | {key(r) for r in high}
    amb = {key(r) for r in ref_b if abs(r["snr"] - thr) < 1e-4 * thr}
    assert (set(got) ^ want) <= amb
    del dev
