"""Continuous-batching server (paper_2108_05602_amd.serve) on cuda:0.

  * every chunk's result is the same alone and in the mix (bit for bit);
  * in the mix, chunks of different subarrays are in flight together;
  * the concatenated per-chunk candidates of a subarray equal one batch
    search of its whole stream;
  * the HBM budget bounds the admitted chunks (one slot: one in flight) and a
    budget that cannot hold a chunk is refused; nothing is ever dropped.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WS = [1, 2, 4, 8, 16, 32]
CHUNK = 244
N_CHUNKS = 6


def _setup():
    import torch
    specs = [synth.evn_scan(4300 + i, n_st, CHUNK * N_CHUNKS, 8, 32, 1.024e-3, 16e6, 2,
                            width_max=16, n_tones=1)
             for i, n_st in enumerate([3, 4, 5])]
    vis = [torch.from_numpy(s.full()).cuda() for s in specs]
    payloads = [[v[:, k * CHUNK:(k + 1) * CHUNK].contiguous() for k in range(N_CHUNKS)] for v in vis]
    subs = [dict(s.desc(), n_ap=CHUNK) for s in specs]
    return specs, vis, payloads, subs


def _fields(c):
    return [tuple(r[f] for f in ("baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr"))
            for r in c]


def _serve(subs, payloads, schedule, **kw):
    from paper_2108_05602_amd.serve import FringeServer, run_schedule
    srv = FringeServer(subs, WS, snr_threshold=4.5, **kw)
    try:
        stats = run_schedule(srv, schedule, payloads)
    finally:
        srv.close()
    return stats


def test_alone_equals_mix_and_overlap():
    from paper_2108_05602_amd.serve import poisson_schedule
    specs, vis, payloads, subs = _setup()
    alone = _serve(subs[:1], payloads[:1], [(0.0, 0, k) for k in range(N_CHUNKS)])
    a_by_seq = {r.seq: r for r in alone.results}
    mix = _serve(subs, payloads, poisson_schedule(3, N_CHUNKS, 2000.0, seed=1))
    assert len(mix.results) == 3 * N_CHUNKS
    for r in mix.results:
        if r.sub == 0:
            assert _fields(r.candidates) == _fields(a_by_seq[r.seq].candidates), r.seq
            assert r.n_windows == a_by_seq[r.seq].n_windows
    assert mix.max_inflight >= 2
    s = mix.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_stream_candidates_equal_batch():
    import torch

    import paper_2108_05602_amd as F
    specs, vis, payloads, subs = _setup()
    stats = _serve(subs, payloads, [(0.0, s, k) for s in range(3) for k in range(N_CHUNKS)])
    for s in range(3):
        got = sorted(tuple(int(c[f]) for f in ("baseline", "window_ap", "t_start"))
                     for r in stats.results if r.sub == s for c in r.candidates)
        with F.Plan([specs[s].desc()], WS, snr_threshold=4.5) as p:
            p.search([vis[s].data_ptr()], torch.cuda.current_stream().cuda_stream)
            want = sorted(tuple(int(c[f]) for f in ("baseline", "window_ap", "t_start"))
                          for c in p.candidates())
        assert got == want


def test_admission_budget():
    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.serve import FringeServer, poisson_schedule
    specs, vis, payloads, subs = _setup()
    plan_bytes = 0
    for s in subs:
        with F.Plan([s], WS, snr_threshold=4.5, flags=F.FRINGE_STREAMING) as p:
            plan_bytes += p.info()["device_bytes"]
    chunk_bytes = max(s["n_baselines"] * CHUNK * 256 * 8 for s in subs)
    one = _serve(subs, payloads, poisson_schedule(3, N_CHUNKS, 5000.0, seed=2),
                 hbm_budget_bytes=plan_bytes + chunk_bytes + chunk_bytes // 2)
    assert one.max_inflight == 1 and len(one.results) == 3 * N_CHUNKS
    with pytest.raises(MemoryError):
        FringeServer(subs, WS, snr_threshold=4.5, hbm_budget_bytes=plan_bytes + chunk_bytes // 2)


def test_batch_server_equals_per_subarray_server():
    """One launch per step over every waiting subarray (FringeBatchServer)
    gives every chunk the same candidates, bit for bit, and the same window
    count as the per-subarray server."""
    from paper_2108_05602_amd.serve import FringeBatchServer, poisson_schedule, run_schedule
    specs, vis, payloads, subs = _setup()
    print("case: batched server vs per-subarray server, 3 subarrays x 6 chunks", flush=True)
    sched = poisson_schedule(3, N_CHUNKS, 2000.0, seed=3)
    ref = {(r.sub, r.seq): r for r in _serve(subs, payloads, sched).results}
    srv = FringeBatchServer(subs, WS, snr_threshold=4.5)
    try:
        got = run_schedule(srv, sched, payloads)
    finally:
        srv.close()
    assert len(got.results) == 3 * N_CHUNKS
    assert got.max_inflight >= 2
    for r in got.results:
        q = ref[(r.sub, r.seq)]
        assert _fields(r.candidates) == _fields(q.candidates), (r.sub, r.seq)
        assert r.n_windows == q.n_windows
    # a subarray's chunks come back in order
    for s in range(3):
        seqs = [r.seq for r in got.results if r.sub == s]
        assert seqs == sorted(seqs)
