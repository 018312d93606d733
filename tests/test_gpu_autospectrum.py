"""Auto-spectrum amplitude normalisation on cuda:0 (fringe_autospectrum_gains,
then fringe_set_gains) against the CPU reference (autospectrum_gains, then
the search of the calibrated data): the device gains equal the reference's
to float rounding, alone and combined in place with calibration gains; the
searches' records agree window by window (peak bins exact, amp / SNR /
energy to 1e-4) on a scan whose stations have their own bandpasses, and a
bandpass-shaped noise-free fringe comes back to the on-grid closed form."""

import math

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import synth
from fringe_testlib import compare_candidates, compare_windows, oracle_table

pytestmark = pytest.mark.gpu


def _device_gains(auto, pairs, n_freq, gains_in=None):
    import torch

    from paper_2108_05602_amd import binding as B
    a = torch.from_numpy(np.ascontiguousarray(auto, dtype=np.float32)).cuda()
    pr = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32)).cuda()
    if gains_in is None:
        out = torch.empty((len(pairs), n_freq), dtype=torch.complex64, device="cuda")
        gin = 0
    else:
        out = torch.from_numpy(np.ascontiguousarray(gains_in, dtype=np.complex64)).cuda()
        gin = out.data_ptr()   # in place
    B.fringe_autospectrum_gains(a.data_ptr(), auto.shape[0], auto.shape[1], n_freq,
                                pr.data_ptr(), len(pairs), gin, out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out


def test_gains_equal_reference():
    print("case: auto-spectrum gains vs reference", flush=True)
    rng = np.random.default_rng(71)
    n_st, n_spec, f = 5, 37, 256
    pairs = synth.baseline_pairs(n_st)
    auto = rng.uniform(0.2, 3.0, (n_st, n_spec, f)).astype(np.float32)
    auto[3, :, 40:44] = 0.0
    want = fo.autospectrum_gains(auto, pairs)
    got = _device_gains(auto, pairs, f).cpu().numpy()
    assert np.allclose(got.real, want, rtol=2e-7, atol=0) and np.all(got.imag == 0)
    assert np.all(got[[b for b, (i, j) in enumerate(pairs) if 3 in (i, j)]][:, 40:44] == 0)
    cal = (rng.uniform(0.5, 1.5, (len(pairs), f)) *
           np.exp(1j * rng.uniform(0, 2 * np.pi, (len(pairs), f)))).astype(np.complex64)
    got2 = _device_gains(auto, pairs, f, gains_in=cal).cpu().numpy()
    assert np.allclose(got2, cal * want, rtol=5e-7, atol=0)


def test_search_with_normalisation_matches_reference():
    import paper_2108_05602_amd as F
    from fringe_testlib import run_gpu
    print("case: normalised search vs reference (bandpassed stations)", flush=True)
    spec = synth.evn_scan(4311, 4, 900, 8, 32, 1.024e-3, 16e6, 3, width_max=16, n_tones=1)
    v = spec.full()
    pairs = synth.baseline_pairs(spec.n_stations)
    rng = np.random.default_rng(5)
    bp = rng.uniform(0.4, 1.8, (spec.n_stations, spec.n_freq))
    shaped = v * np.stack([bp[i] * bp[j] for i, j in pairs])[:, None, :].reshape(
        len(pairs), 1, spec.n_if, spec.n_chan)
    shaped = shaped.astype(np.complex64)
    auto = np.stack([np.tile(bp[s] ** 2, (16, 1)) * rng.uniform(0.9, 1.1, (16, spec.n_freq))
                     for s in range(spec.n_stations)]).astype(np.float32)
    g = _device_gains(auto, pairs, spec.n_freq)
    ws, thr = [1, 2, 4, 8, 16, 32], 4.5
    d = spec.desc()
    import torch
    dev = torch.from_numpy(shaped).cuda()
    with F.Plan([d], ws, pad_freq=4, pad_time=2, snr_threshold=thr) as plan:
        plan.set_gains(0, g.data_ptr())
        plan.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        table = plan.windows(np.arange(plan.info()["n_windows"]))
        cands = plan.candidates()
    ref_g = fo.autospectrum_gains(auto, pairs)
    ref = oracle_table([shaped], [d], ws, 4, 2, thr, gains=[ref_g])
    cal = fo.calibrate(shaped.reshape(len(pairs), spec.n_ap, -1), ref_g)
    n_amb = compare_windows(table, ref, lambda s, b: cal[b], 4, 2, "normalised")
    compare_candidates(cands, ref, thr, "normalised")
    assert n_amb <= max(2, len(ref) // 1000)


def test_bandpassed_fringe_closed_form():
    import torch

    import paper_2108_05602_amd as F
    print("case: bandpassed noise-free fringe", flush=True)
    w, n_if, n_chan, kt, kf = 8, 4, 16, 5, 37
    f = n_if * n_chan
    mt, mf = 2 * w, 4 * f
    pairs = [(0, 1), (0, 2), (1, 2)]
    rng = np.random.default_rng(9)
    bp = rng.uniform(0.3, 2.0, (3, f))
    u = np.arange(w)[:, None]
    ff = np.arange(f)[None, :]
    fr = np.exp(2j * np.pi * (kt * u / mt + kf * ff / mf))
    vis = np.stack([bp[i] * bp[j] * fr for i, j in pairs]).reshape(3, w, n_if, n_chan)
    vis = vis.astype(np.complex64)
    auto = np.repeat((bp ** 2)[:, None, :], 3, axis=1).astype(np.float32)
    g = _device_gains(auto, pairs, f)
    d = dict(n_baselines=3, n_ap=w, n_if=n_if, n_chan=n_chan, ap_seconds=1.0, chan_width_hz=1.0)
    dev = torch.from_numpy(vis).cuda()
    with F.Plan([d], [w], pad_freq=4, pad_time=2, snr_threshold=1.0) as plan:
        plan.set_gains(0, g.data_ptr())
        plan.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        t = plan.windows(np.arange(3))
    for b in range(3):
        assert (int(t["k_rate"][b]), int(t["k_delay"][b])) == (kt, kf)
        assert float(t["amp"][b]) == pytest.approx(w * f, rel=2e-5)
        assert float(t["snr"][b]) == pytest.approx(math.sqrt(w * f), rel=2e-5)
