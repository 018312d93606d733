"""The library's native server (fringe_server_*, FringeNativeServer) on cuda:0.

  * every chunk's candidates equal those of the Python server's (the same
    streaming plans), bit for bit, on a Poisson mix of three subarrays, and
    each subarray's results come in chunk order;
  * with dedispersion shifts, the candidates of a streaming plan with the
    same shifts; shifts after the first submission are refused;
  * max_inflight = 1 serialises the subarrays (first come, first served)
    and loses nothing; timestamps are ordered (submit <= launch <= done).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WS = [1, 2, 4, 8, 16, 32]
CHUNK = 244
N_CHUNKS = 6
FIELDS = ("baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy")


def _setup():
    import torch
    specs = [synth.evn_scan(4700 + i, n_st, CHUNK * N_CHUNKS, 8, 32, 1.024e-3, 16e6, 2,
                            width_max=16, n_tones=1)
             for i, n_st in enumerate([3, 4, 5])]
    vis = [torch.from_numpy(s.full()).cuda() for s in specs]
    payloads = [[v[:, k * CHUNK:(k + 1) * CHUNK].contiguous() for k in range(N_CHUNKS)] for v in vis]
    subs = [dict(s.desc(), n_ap=CHUNK) for s in specs]
    torch.cuda.synchronize()
    return specs, payloads, subs


def _same(a, b, label):
    assert len(a) == len(b), label
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (label, f)


def _serve(cls, subs, payloads, sched, **kw):
    from paper_2108_05602_amd.serve import run_schedule
    srv = cls(subs, WS, snr_threshold=4.5, **kw)
    try:
        stats = run_schedule(srv, sched, payloads)
    finally:
        srv.close()
    return stats


def test_native_equals_python_server():
    from paper_2108_05602_amd.serve import FringeNativeServer, FringeServer, poisson_schedule
    print("case: native vs Python server, 3 subarrays x 6 chunks, Poisson", flush=True)
    specs, payloads, subs = _setup()
    sched = poisson_schedule(3, N_CHUNKS, 1500.0, seed=3)
    py = _serve(FringeServer, subs, payloads, sched, time_chunk=64)
    nat = _serve(FringeNativeServer, subs, payloads, sched, time_chunk=64)
    assert len(nat.results) == len(py.results) == 3 * N_CHUNKS
    p_by = {(r.sub, r.seq): r for r in py.results}
    for s in range(3):
        seqs = [r.seq for r in nat.results if r.sub == s]
        assert seqs == list(range(N_CHUNKS)), (s, seqs)
    for r in nat.results:
        q = p_by[(r.sub, r.seq)]
        _same(r.candidates, q.candidates, f"chunk {r.sub}/{r.seq}")
        assert r.n_windows == q.n_windows
        assert r.done >= r.arrival
    s = nat.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_native_server_shifts_and_serial():
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd import binding as B
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    from paper_2108_05602_amd.serve import FringeNativeServer
    print("case: native server with shifts; max_inflight 1", flush=True)
    specs, payloads, subs = _setup()
    sh = []
    for sd in subs:
        f = channel_freqs_hz(1.6e9, sd["n_if"], sd["n_chan"], sd["chan_width_hz"])
        sh.append(torch.from_numpy(dm_shifts(150.0, f, sd["ap_seconds"])).cuda())
    burst = [(0.0, s, k) for s in range(3) for k in range(N_CHUNKS)]
    ded = _serve(FringeNativeServer, subs, payloads, burst, shifts=sh)
    got = {(r.sub, r.seq): r.candidates for r in ded.results}
    st = torch.cuda.current_stream().cuda_stream
    for s in range(3):
        with F.Plan([subs[s]], WS, snr_threshold=4.5, flags=F.FRINGE_STREAMING) as p:
            p.set_shifts(0, sh[s].data_ptr())
            for k in range(N_CHUNKS):
                p.search([payloads[s][k].data_ptr()], st)
                _same(got[(s, k)], p.candidates(), f"dedispersed {s}/{k}")
    # shifts once chunks have been submitted: refused
    h = B.fringe_server_create(subs, WS, snr_threshold=4.5)
    try:
        B.fringe_server_submit(h, 0, 0, payloads[0][0].data_ptr())
        with pytest.raises(F.FringeError) as e:
            B.fringe_server_set_shifts(h, 0, sh[0].data_ptr())
        assert e.value.code == B.FRINGE_E_STATE
    finally:
        B.fringe_server_destroy(h)
    # one chunk at a time over all subarrays: first come, first served
    h = B.fringe_server_create(subs, WS, snr_threshold=4.5, max_inflight=1)
    try:
        for k in range(N_CHUNKS):
            for s in range(3):
                B.fringe_server_submit(h, s, 100 * s + k, payloads[s][k].data_ptr())
        res = []
        while len(res) < 3 * N_CHUNKS:
            r, _ = B.fringe_server_poll(h)
            res += r
        assert B.fringe_server_pending(h) == 0
    finally:
        B.fringe_server_destroy(h)
    assert [r["tag"] for r in res] == [100 * s + k for k in range(N_CHUNKS) for s in range(3)]
    for a, b in zip(res, res[1:]):
        assert b["t_launch_ns"] >= a["t_done_ns"] - 1_000_000   # serial (the worker's order)
    for r in res:
        assert r["status"] == 0 and r["t_submit_ns"] <= r["t_launch_ns"] <= r["t_done_ns"]
