"""HIP path vs the CPU reference, through the C ABI, on cuda:0.

Sizes here are ones the reference finishes in seconds while still spanning
several bin blocks, time chunks and ragged tails; the full-size EVN-like
scan is covered by tests/test_gpu_fullsize.py.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import synth
from fringe_testlib import compare_candidates, compare_windows, oracle_table, run_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_2108_05602_amd as F
    F.load()
    torch.cuda.init()


def _flat(v):
    return v.reshape(v.shape[0], v.shape[1], -1)


def _scan_run(spec, params, **kw):
    v = spec.full()
    d = spec.desc()
    plan, table, cands = run_gpu([d], [v], params["window_aps"], params["pad_freq"],
                                 params["pad_time"], params["snr_threshold"], **kw)
    ref = oracle_table([v], [d], params["window_aps"], params["pad_freq"], params["pad_time"],
                       params["snr_threshold"])
    return v, plan, table, cands, ref


def test_c1_full_parity():
    print("case: C1 noisy, seed 0", flush=True)
    spec = synth.c1()
    v, plan, table, cands, ref = _scan_run(spec, synth.C1_PARAMS)
    fv = _flat(v)
    compare_windows(table, ref, lambda s, b: fv[b], 4, 2, "C1")
    compare_candidates(cands, ref, 3.0, "C1")
    plan.close()


def test_c1_noise_free_closed_form():
    print("case: C1 noise-free", flush=True)
    gold = json.load(open(os.path.join(GOLDEN, "c1_noise_free.json")))
    spec = synth.c1(noise=False)
    v, plan, table, cands, ref = _scan_run(spec, synth.C1_PARAMS)
    assert [int(c) for c in cands["t_start"]] == [g["t_start"] for g in gold["candidates"]]
    for c, g in zip(cands, gold["candidates"]):
        assert (int(c["k_rate"]), int(c["k_delay"])) == (g["k_rate"], g["k_delay"])
        assert c["amp"] == pytest.approx(g["amp"], rel=1e-5)
        assert c["snr"] == pytest.approx(g["snr"], rel=1e-5)
    rest = table[~np.isin(table["t_start"], cands["t_start"])]
    assert np.all(rest["amp"] == 0) and np.all(rest["snr"] == 0)
    assert np.all(rest["k_rate"] == 0) and np.all(rest["k_delay"] == 0)
    plan.close()


def test_grid_dump_brute_force_and_parseval():
    """Every grid bin of every window against the direct DFT (P7), and
    Parseval on the GPU's own grid (P2)."""
    import paper_2108_05602_amd as F
    print("case: C1 grid dump", flush=True)
    spec = synth.c1()
    v = spec.full()
    fv = _flat(v)
    plan, table, _ = run_gpu([spec.desc()], [v], [4], 4, 2, 3.0, flags=F.FRINGE_DUMP_GRID)
    y = fo.delay_spectra(fv[0], 4)
    for i, row in enumerate(table):
        t0 = int(row["t_start"])
        g = plan.grid(i, 8, 128)
        ref = fo.window_grid(y, t0, 4, 2)
        scale = np.abs(ref).max()
        assert np.allclose(g, ref, rtol=0, atol=2e-6 * scale), f"window {t0}"
        e = float(np.sum(np.abs(fv[0, t0:t0 + 4]).astype(np.float64) ** 2))
        assert float(np.sum(np.abs(g.astype(np.complex128)) ** 2)) == pytest.approx(8 * 128 * e, rel=1e-5)
    plan.close()


SHAPES = [
    # (n_bl, T, n_if, n_chan, windows, pad_f, pad_t)
    (2, 300, 4, 4, [1, 2, 4, 8, 16, 32], 4, 2),        # M_f = 64: one bin block
    (1, 517, 8, 32, [1, 2, 4, 8, 16, 32], 4, 2),       # C2 channel layout, ragged tail
    (3, 200, 2, 16, [2, 8], 2, 2),                     # pad_freq 2, sparse lengths
    (2, 130, 16, 16, [1, 4, 16], 1, 1),                # no padding at all
    (1, 260, 1, 64, [64], 4, 2),                       # W = 64 only (S = 4 sub-transforms)
    (1, 300, 8, 8, [1, 128], 4, 2),                    # W = 128 (S = 8), T not a multiple
    (2, 1100, 4, 16, [1, 2, 4, 8, 16, 32], 4, 2),      # several time chunks per wave
    (1, 40, 32, 32, [2, 4, 8], 4, 1),                  # M_f = 4096, pad_time 1
    (2, 1400, 4, 16, [64, 128], 4, 1),                 # W = 128 at pad_time 1, two time chunks
    (1, 2200, 2, 32, [128], 4, 2),                     # W = 128 alone, three chunks, ragged tail
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"s{i}" for i in range(len(SHAPES))])
def test_random_shapes(shape):
    nb, t, n_if, n_chan, ws, pf, pt = shape
    print(f"case: random shape {shape}", flush=True)
    rng = np.random.default_rng([77, nb, t, n_if, n_chan])
    v = (rng.standard_normal((nb, t, n_if, n_chan)) +
         1j * rng.standard_normal((nb, t, n_if, n_chan))).astype(np.complex64)
    # a strong on-grid fringe so that some windows are clear candidates
    f = np.arange(n_if * n_chan)
    v[0, t // 3:t // 3 + 5] += (0.8 * np.exp(2j * np.pi * 0.17 * f)).reshape(n_if, n_chan).astype(np.complex64)
    d = dict(n_baselines=nb, n_ap=t, n_if=n_if, n_chan=n_chan, ap_seconds=1e-3,
             chan_width_hz=1e6)
    thr = 4.0
    plan, table, cands = run_gpu([d], [v], ws, pf, pt, thr)
    ref = oracle_table([v], [d], ws, pf, pt, thr)
    fv = _flat(v)
    n_amb = compare_windows(table, ref, lambda s, b: fv[b], pf, pt, str(shape))
    compare_candidates(cands, ref, thr, str(shape))
    assert n_amb <= max(2, len(ref) // 1000)
    plan.close()


def test_several_scans_in_one_plan():
    """Uneven scans in one plan give the per-scan results (P11, batched ==
    per-scan) with scan indices and window ids in order."""
    print("case: three uneven scans", flush=True)
    ws, pf, pt, thr = [1, 2, 4, 8], 4, 2, 4.0
    specs = [synth.evn_scan(900 + i, n_st, n_ap, n_if, n_chan, 1.024e-3, 16e6, 2, width_max=8)
             for i, (n_st, n_ap, n_if, n_chan) in
             enumerate([(3, 150, 8, 16), (2, 97, 4, 16), (4, 64, 8, 8)])]
    vis = [s.full() for s in specs]
    descs = [s.desc() for s in specs]
    plan, table, cands = run_gpu(descs, vis, ws, pf, pt, thr)
    ref = oracle_table(vis, descs, ws, pf, pt, thr)
    assert np.array_equal(table["scan"], ref["scan"])
    compare_windows(table, ref, lambda s, b: _flat(vis[s])[b], pf, pt, "multi-scan")
    compare_candidates(cands, ref, thr, "multi-scan")
    # batched equals separate plans, field for field
    for s in range(3):
        p1, t1, c1 = run_gpu([descs[s]], [vis[s]], ws, pf, pt, thr)
        sub = table[table["scan"] == s]
        for k in ("baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy"):
            assert np.array_equal(sub[k], t1[k]), (s, k)
        p1.close()
    plan.close()


def test_edge_cases():
    print("case: edges", flush=True)
    base = dict(n_baselines=1, n_if=2, n_chan=32, ap_seconds=1e-3, chan_width_hz=1e6)
    # data shorter than every window: no windows, no candidates
    v = np.ones((1, 3, 2, 32), np.complex64)
    plan, table, cands = run_gpu([dict(base, n_ap=3)], [v], [4, 8], 4, 2, 1.0)
    assert plan.info()["n_windows"] == 0 and len(cands) == 0
    plan.close()
    # all-zero data: peak (0, 0), amplitude and SNR 0, no candidates even at threshold 0
    z = np.zeros((1, 40, 2, 32), np.complex64)
    plan, table, cands = run_gpu([dict(base, n_ap=40)], [z], [1, 2, 4, 8], 4, 2, 0.0)
    assert len(cands) == 0
    assert np.all(table["amp"] == 0) and np.all(table["snr"] == 0)
    assert np.all(table["k_rate"] == 0) and np.all(table["k_delay"] == 0)
    plan.close()
    # one AP, one-AP windows: the two identical rate rows tie, rate bin 0 wins
    rng = np.random.default_rng(1)
    one = (rng.standard_normal((1, 1, 2, 32)) + 1j * rng.standard_normal((1, 1, 2, 32))).astype(np.complex64)
    plan, table, cands = run_gpu([dict(base, n_ap=1)], [one], [1], 4, 2, 0.0)
    ref = oracle_table([one], [dict(base, n_ap=1)], [1], 4, 2, 0.0)
    assert len(table) == 1 and table["k_rate"][0] == 0
    compare_windows(table, ref, lambda s, b: _flat(one)[b], 4, 2, "one AP")
    plan.close()
    # window exactly the data length
    w = (rng.standard_normal((1, 16, 2, 32)) + 1j * rng.standard_normal((1, 16, 2, 32))).astype(np.complex64)
    plan, table, cands = run_gpu([dict(base, n_ap=16)], [w], [16], 4, 2, 0.0)
    ref = oracle_table([w], [dict(base, n_ap=16)], [16], 4, 2, 0.0)
    compare_windows(table, ref, lambda s, b: _flat(w)[b], 4, 2, "W = T")
    plan.close()


def test_candidate_capacity():
    """Overflow is counted, not lost: the true total is reported and the
    first candidates in key order are kept."""
    import paper_2108_05602_amd as F
    from paper_2108_05602_amd import binding as B
    print("case: capacity", flush=True)
    spec = synth.c1()
    v = spec.full()
    full_plan, _, full = run_gpu([spec.desc()], [v], [4], 4, 2, 3.0, all_windows=False)
    n = len(full)
    assert n >= 3
    import torch
    t = torch.from_numpy(v).cuda()
    p = F.Plan([spec.desc()], [4], pad_freq=4, pad_time=2, snr_threshold=3.0, max_candidates=2)
    p.search([t.data_ptr()], torch.cuda.current_stream().cuda_stream)
    rc, total, recs = B.candidates_get_raw(p.handle, 10, 2)
    assert rc == B.FRINGE_E_CAPACITY and total == n and len(recs) == 2
    assert np.array_equal(recs["t_start"], full["t_start"][:2])
    rc, total, recs = B.candidates_get_raw(full_plan.handle, 1, 1 << 16)
    assert rc == B.FRINGE_E_CAPACITY and total == n and recs["t_start"][0] == full["t_start"][0]
    rc, total, recs = B.candidates_get_raw(full_plan.handle, n, 1 << 16)
    assert rc == B.FRINGE_OK and total == n
    p.close()
    full_plan.close()


def test_errors_on_device():
    import paper_2108_05602_amd as F
    from paper_2108_05602_amd import binding as B
    d = dict(n_baselines=1, n_ap=64, n_if=2, n_chan=16, ap_seconds=1.0, chan_width_hz=1.0)
    p = F.Plan([d], [4], pad_freq=4, pad_time=2, snr_threshold=3.0)
    with pytest.raises(F.FringeError) as e:
        p.candidates()
    assert e.value.code == B.FRINGE_E_STATE
    with pytest.raises(F.FringeError) as e:
        p.search([0])
    assert e.value.code == B.FRINGE_E_INVALID
    with pytest.raises(F.FringeError):
        p.window_id(0, 0, 4, 3)          # 3 is not a start of a 4-AP window
    assert p.window_id(0, 0, 4, 60) == 30
    p.close()
    with pytest.raises(F.FringeError) as e:
        F.Plan([d], [4], hbm_budget_bytes=1024)
    assert e.value.code == B.FRINGE_E_NOMEM


def test_evn_mini_full_table():
    """The EVN-like recipe at 6 baselines x 3000 APs: every window."""
    print("case: EVN-like mini (6 BL x 3000 AP)", flush=True)
    spec = synth.c2(seed=11, n_stations=4, n_ap=3000, n_pulses=6, n_tones=2)
    v, plan, table, cands, ref = _scan_run(spec, synth.C2_PARAMS)
    fv = _flat(v)
    n_amb = compare_windows(table, ref, lambda s, b: fv[b], 4, 2, "EVN mini")
    compare_candidates(cands, ref, synth.C2_PARAMS["snr_threshold"], "EVN mini")
    print(f"windows {len(ref)} candidates {len(cands)} ambiguous {n_amb}", flush=True)
    plan.close()


def test_dense_mini_sampled():
    """The large-dense recipe (16 IF x 64 chan, W up to 128) on 3 baselines
    x 700 APs: every candidate and 300 sampled windows against the reference."""
    print("case: dense mini (3 BL x 700 AP, F = 1024)", flush=True)
    spec = synth.c5(seed=15, n_stations=3, n_ap=700, n_pulses=4, n_bursts=2)
    p = synth.C5_PARAMS
    v = spec.full()
    d = spec.desc()
    plan, table, cands = run_gpu([d], [v], p["window_aps"], p["pad_freq"], p["pad_time"],
                                 p["snr_threshold"])
    fv = _flat(v)
    rng = np.random.default_rng(5)
    idx = set(rng.choice(len(table), 300, replace=False).tolist())
    idx |= set(np.nonzero(table["snr"] > 0.9 * p["snr_threshold"])[0].tolist())
    idx = sorted(idx)
    rows = []
    for i in idx:
        g = table[i]
        r = fo.search_window(fv[g["baseline"]], int(g["t_start"]), int(g["window_ap"]),
                             p["pad_freq"], p["pad_time"])
        m_f = p["pad_freq"] * spec.n_freq
        m_t = p["pad_time"] * int(g["window_ap"])
        rows.append((0, g["baseline"], g["window_ap"], g["t_start"], r.k_rate, r.k_delay,
                     r.amp, r.snr, r.energy,
                     fo.signed_bin(r.k_delay, m_f) / (m_f * spec.chan_width_hz),
                     fo.signed_bin(r.k_rate, m_t) / (m_t * spec.ap_seconds), r.margin))
    ref = np.array(rows, dtype=fo.TABLE_DTYPE)
    compare_windows(table[idx], ref, lambda s, b: fv[b], p["pad_freq"], p["pad_time"], "dense")
    # every window that could be a candidate was re-computed by the reference
    ref_c = ref[ref["snr"] > p["snr_threshold"]]
    got = {(int(c["baseline"]), int(c["window_ap"]), int(c["t_start"])) for c in cands}
    want = {(int(c["baseline"]), int(c["window_ap"]), int(c["t_start"])) for c in ref_c}
    near = {(int(c["baseline"]), int(c["window_ap"]), int(c["t_start"])) for c in ref
            if abs(c["snr"] - p["snr_threshold"]) < 1e-4 * p["snr_threshold"]}
    assert (got ^ want) <= near
    plan.close()


def test_plain_path_equals_batched():
    """One window per launch (FRINGE_PLAIN) gives the batched records."""
    import paper_2108_05602_amd as F
    print("case: plain vs batched", flush=True)
    spec = synth.c2(seed=12, n_stations=3, n_ap=300, n_pulses=3, n_tones=1)
    v = spec.full()
    p = synth.C2_PARAMS
    args = ([spec.desc()], [v], p["window_aps"], p["pad_freq"], p["pad_time"], p["snr_threshold"])
    pb, tb, cb = run_gpu(*args)
    pp, tp, cp = run_gpu(*args, flags=F.FRINGE_PLAIN)
    for k in ("baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy"):
        assert np.array_equal(tb[k], tp[k]), k
    assert np.array_equal(cb["t_start"], cp["t_start"])
    pb.close()
    pp.close()


def test_batched_uneven_scans_one_launch():
    """Scans of uneven baselines, lengths and channel counts (8/16 IF x
    16/32/64 chan, windows up to 64 APs) searched by one plan: one fused
    launch per fold class of their bands (the kernel instantiation each
    band needs).  Equal to per-scan plans field by field, and to the
    reference on sampled windows; a tight HBM budget splits the scans into
    several groups with the same results."""
    import paper_2108_05602_amd as F
    print("case: batched uneven scans", flush=True)
    specs = synth.c3(n_scans=6, max_ap=600, max_stations=5)
    p = synth.C3_PARAMS
    vis = [s.full() for s in specs]
    descs = [s.desc() for s in specs]
    args = (p["window_aps"], p["pad_freq"], p["pad_time"], p["snr_threshold"])
    plan, table, cands = run_gpu(descs, vis, *args, flags=F.FRINGE_PROFILE)
    prof = plan.profile()
    classes = {min(16, max(4, 1 << math.ceil(math.log2(max(1, s.n_freq // 64))))) for s in specs}
    assert len(classes) > 1, "the sample should mix fold classes"
    assert prof["rate_launches"] == len(classes) == prof["finalize_launches"], prof
    for s in range(len(specs)):
        p1, t1, _ = run_gpu([descs[s]], [vis[s]], *args)
        sub = table[table["scan"] == s]
        for k in ("baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy"):
            assert np.array_equal(sub[k], t1[k]), (s, k)
        p1.close()
    need = plan.info()["device_bytes"] - plan.info()["scratch_bytes"]
    tight, t2, c2 = run_gpu(descs, vis, *args, flags=F.FRINGE_PROFILE,
                            max_candidates=1 << 16)
    tight.close()
    small = F.Plan(descs, p["window_aps"], pad_freq=p["pad_freq"], pad_time=p["pad_time"],
                   snr_threshold=p["snr_threshold"], flags=F.FRINGE_PROFILE,
                   hbm_budget_bytes=need + plan.info()["scratch_bytes"] // 3)
    import torch
    tens = [torch.from_numpy(v).cuda() for v in vis]
    small.search([t.data_ptr() for t in tens], torch.cuda.current_stream().cuda_stream)
    ts = small.windows(np.arange(small.info()["n_windows"]))
    assert small.profile()["rate_launches"] > 1
    for k in ("scan", "baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr"):
        assert np.array_equal(ts[k], table[k]), k
    small.close()
    # reference on samples of every scan
    rng = np.random.default_rng(8)
    idx = np.sort(rng.choice(len(table), 200, replace=False))
    rows = []
    for i in idx:
        g = table[i]
        spec = specs[int(g["scan"])]
        fv = vis[int(g["scan"])].reshape(spec.n_baselines, spec.n_ap, -1)
        r = fo.search_window(fv[g["baseline"]], int(g["t_start"]), int(g["window_ap"]),
                             p["pad_freq"], p["pad_time"])
        m_f = p["pad_freq"] * spec.n_freq
        m_t = p["pad_time"] * int(g["window_ap"])
        rows.append((g["scan"], g["baseline"], g["window_ap"], g["t_start"], r.k_rate, r.k_delay,
                     r.amp, r.snr, r.energy,
                     fo.signed_bin(r.k_delay, m_f) / (m_f * spec.chan_width_hz),
                     fo.signed_bin(r.k_rate, m_t) / (m_t * spec.ap_seconds), r.margin))
    ref = np.array(rows, dtype=fo.TABLE_DTYPE)

    def xb(s, b):
        sp = specs[s]
        return vis[s].reshape(sp.n_baselines, sp.n_ap, -1)[b]
    compare_windows(table[idx], ref, xb, p["pad_freq"], p["pad_time"], "batched")
    plan.close()
