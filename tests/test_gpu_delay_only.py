"""The delay-only search (FRINGE_DELAY_ONLY) on cuda:0 against the CPU
reference's delay-only search, through the C ABI.

Per window: the APs summed coherently, one zero-padded delay transform, the
peak over the delay axis and E = the mean power over it.  Covered: the 64-AP
workload in full (noisy, and noise-free against its closed form), random
shapes with ragged tails and every supported window length, an EVN-like
scan slice, several uneven scans in one plan, streamed == batch, and the
one-window-per-launch path == batched.
"""

import math

import numpy as np
import pytest

import synth
from fringe_testlib import compare_candidates, compare_windows, oracle_table, run_gpu

pytestmark = pytest.mark.gpu


def _flat(v):
    return v.reshape(v.shape[0], v.shape[1], -1)


def _key(r):
    return (int(r["scan"]), int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))


def _flags():
    import paper_2108_05602_amd as F
    return F.FRINGE_DELAY_ONLY


def test_c1_delay_only():
    print("case: C1 delay-only, noisy and noise-free", flush=True)
    for noise in (True, False):
        spec = synth.c1(noise=noise)
        v = spec.full()
        d = spec.desc()
        plan, table, cands = run_gpu([d], [v], [4], 4, 2, 3.0, flags=_flags())
        ref = oracle_table([v], [d], [4], 4, 2, 3.0, delay_only=True)
        fv = _flat(v)
        compare_windows(table, ref, lambda s, b: fv[b], 4, 2, f"C1 noise={noise}")
        compare_candidates(cands, ref, 3.0, f"C1 noise={noise}")
        assert np.all(table["k_rate"] == 0) and np.all(table["rate_hz"] == 0.0)
        if not noise:
            # closed form: SNR = sqrt(F) for every window holding fringe APs
            assert [int(t) for t in cands["t_start"]] == [18, 20, 22]
            assert np.allclose(cands["snr"], math.sqrt(32), rtol=1e-5)
            assert cands["amp"][1] == pytest.approx(16 / math.sin(math.pi / 8), rel=1e-5)
        plan.close()


SHAPES = [
    # (n_bl, T, n_if, n_chan, windows, pad_f)
    (2, 300, 4, 4, [1, 2, 4, 8, 16, 32], 4),
    (1, 517, 8, 32, [1, 2, 4, 8, 16, 32], 4),
    (3, 200, 2, 16, [2, 8], 2),
    (2, 130, 16, 16, [1, 4, 16], 1),
    (1, 260, 1, 64, [64], 4),
    (2, 1100, 4, 16, [1, 2, 4, 8, 16, 32, 64], 4),
    (1, 90, 32, 32, [2, 4, 8], 4),
    (2, 333, 16, 32, [1, 2, 4, 8, 16, 32], 4),
    (1, 275, 8, 64, [1, 4, 16, 64], 2),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"s{i}" for i in range(len(SHAPES))])
def test_random_shapes_delay_only(shape):
    nb, t, n_if, n_chan, ws, pf = shape
    print(f"case: delay-only shape {shape}", flush=True)
    rng = np.random.default_rng([91, nb, t, n_if, n_chan])
    v = (rng.standard_normal((nb, t, n_if, n_chan)) +
         1j * rng.standard_normal((nb, t, n_if, n_chan))).astype(np.complex64)
    f = np.arange(n_if * n_chan)
    v[0, t // 3:t // 3 + 5] += (0.8 * np.exp(2j * np.pi * 0.17 * f)).reshape(n_if, n_chan).astype(np.complex64)
    d = dict(n_baselines=nb, n_ap=t, n_if=n_if, n_chan=n_chan, ap_seconds=1e-3, chan_width_hz=1e6)
    plan, table, cands = run_gpu([d], [v], ws, pf, 2, 4.0, flags=_flags())
    ref = oracle_table([v], [d], ws, pf, 2, 4.0, delay_only=True)
    fv = _flat(v)
    n_amb = compare_windows(table, ref, lambda s, b: fv[b], pf, 2, str(shape))
    compare_candidates(cands, ref, 4.0, str(shape))
    assert n_amb <= max(2, len(ref) // 1000)
    plan.close()


def test_evn_slice_and_uneven_scans_delay_only():
    """An EVN-like slice (pulses and a tone) and uneven scans in one plan."""
    print("case: delay-only EVN slice + uneven scans", flush=True)
    specs = [synth.evn_scan(5001, 4, 1200, 8, 32, 1.024e-3, 16e6, 3, width_max=32, n_tones=1)]
    specs += synth.c3(n_scans=3, max_ap=400, max_stations=4)
    vis = [s.full() for s in specs]
    descs = [s.desc() for s in specs]
    ws = [1, 2, 4, 8, 16, 32, 64]
    plan, table, cands = run_gpu(descs, vis, ws, 4, 2, 4.5, flags=_flags())
    ref = oracle_table(vis, descs, ws, 4, 2, 4.5, delay_only=True)
    fv = [_flat(v) for v in vis]
    compare_windows(table, ref, lambda s, b: fv[s][b], 4, 2, "delay-only multi-scan")
    compare_candidates(cands, ref, 4.5, "delay-only multi-scan")
    assert len(cands) > 0
    plan.close()


def test_streamed_and_plain_equal_batch_delay_only():
    import torch

    import paper_2108_05602_amd as F
    print("case: delay-only streamed / plain vs batch", flush=True)
    spec = synth.evn_scan(5002, 3, 1464, 8, 32, 1.024e-3, 16e6, 2, width_max=16, n_tones=1)
    vis = spec.full()
    desc = spec.desc()
    ws = [1, 2, 4, 8, 16, 32]
    _, batch, bc = run_gpu([desc], [vis], ws, 4, 2, 4.5, flags=F.FRINGE_DELAY_ONLY)
    bmap = {_key(r): r for r in batch}
    fields = ("k_rate", "k_delay", "amp", "snr", "energy", "delay_s", "rate_hz")
    dev = torch.from_numpy(vis).cuda()
    st = torch.cuda.current_stream().cuda_stream
    for chunk in (488, 61):
        got = []
        with F.Plan([dict(desc, n_ap=chunk)], ws, snr_threshold=4.5,
                    flags=F.FRINGE_STREAMING | F.FRINGE_DELAY_ONLY) as p:
            for t0 in range(0, vis.shape[1] - chunk + 1, chunk):
                piece = dev[:, t0:t0 + chunk].contiguous()
                p.search([piece.data_ptr()], st)
                n = p.info()["n_windows"]
                if n:
                    got.append(p.windows(np.arange(n)))
                torch.cuda.synchronize()
        rows = np.concatenate(got)
        n_used = (vis.shape[1] // chunk) * chunk
        assert {_key(r) for r in rows} == {k for k in bmap if k[3] + k[2] <= n_used}
        assert len(rows) == len({_key(r) for r in rows})
        for r in rows:
            b = bmap[_key(r)]
            for f in fields:
                assert r[f] == b[f], (chunk, _key(r), f)
    d300 = dict(desc, n_ap=300)
    sub = np.ascontiguousarray(vis[:, :300])
    _, plain, _ = run_gpu([d300], [sub], ws, 4, 2, 4.5, flags=F.FRINGE_DELAY_ONLY | F.FRINGE_PLAIN)
    _, b300, _ = run_gpu([d300], [sub], ws, 4, 2, 4.5, flags=F.FRINGE_DELAY_ONLY)
    for f in ("baseline", "window_ap", "t_start") + fields:
        assert np.array_equal(plain[f], b300[f]), f


@pytest.mark.parametrize("n_if,n_chan,pf", [(4, 4, 4), (2, 16, 4), (4, 16, 4), (8, 16, 4), (8, 32, 4),
                                            (8, 32, 2), (16, 32, 4), (16, 64, 4)],
                         ids=["F16", "F32", "F64", "F128", "F256", "F256-pad2", "F512", "F1024"])
def test_exact_ties_delay_only(n_if, n_chan, pf):
    """Every delay bin ties exactly: each AP holds one nonzero sample, in
    channel 0, so its delay spectrum is that sample in every bin (the
    transform only adds zeros to it), and so is every window's sum.  The
    peak is then the lowest delay bin, 0, as in the reference, whichever
    wave, class and lane hold the other bins (four classes per wave for the
    bands of up to 256 channels, two above; with 16 and 32 channels at pad
    4 the bins make only one and two classes, and the wave's other classes
    are ghosts that must never win)."""
    nb, t, ws = 2, 300, [1, 2, 4, 8, 16, 32]
    print(f"case: delay-only exact ties, F = {n_if * n_chan}, pad {pf}", flush=True)
    rng = np.random.default_rng([97, n_if, n_chan, pf])
    v = np.zeros((nb, t, n_if, n_chan), np.complex64)
    v[:, :, 0, 0] = (rng.standard_normal((nb, t)) + 1j * rng.standard_normal((nb, t))).astype(np.complex64)
    d = dict(n_baselines=nb, n_ap=t, n_if=n_if, n_chan=n_chan, ap_seconds=1e-3, chan_width_hz=1e6)
    plan, table, _ = run_gpu([d], [v], ws, pf, 2, 3.0, flags=_flags())
    ref = oracle_table([v], [d], ws, pf, 2, 3.0, delay_only=True)
    assert np.all(ref["k_delay"] == 0)
    assert np.all(table["k_delay"] == 0) and np.all(table["delay_s"] == 0.0)
    fv = _flat(v)
    compare_windows(table, ref, lambda s, b: fv[b], pf, 2, f"ties F={n_if * n_chan} pad {pf}")
    plan.close()
