"""Streaming plans (FRINGE_STREAMING) on cuda:0.

A subarray's scan fed chunk by chunk must give, window for window, the
records of one batch search of the whole scan (P11: streamed with any
chunking == batch on the concatenated stream), with absolute start APs,
for chunk lengths that are and are not multiples of the window strides,
including chunks shorter than the longest window.  Each call reports the
windows whose last AP lies in its chunk, so over the stream every window is
reported exactly once.
"""

import numpy as np
import pytest

import synth
from fringe_testlib import compare_windows, oracle_table

pytestmark = pytest.mark.gpu


def _key(r):
    return (int(r["scan"]), int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))


def _batch(desc, vis, ws, thr):
    import torch

    import paper_2108_05602_amd as F
    dev = torch.from_numpy(vis).cuda()
    with F.Plan([desc], ws, pad_freq=4, pad_time=2, snr_threshold=thr) as p:
        p.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        table = p.windows(np.arange(p.info()["n_windows"]))
        cands = p.candidates()
    return table, cands


def _streamed(desc, vis, ws, thr, chunk):
    import torch

    import paper_2108_05602_amd as F
    d = dict(desc, n_ap=chunk)
    dev = torch.from_numpy(vis).cuda()
    rows, cands = [], []
    with F.Plan([d], ws, pad_freq=4, pad_time=2, snr_threshold=thr,
                flags=F.FRINGE_STREAMING) as p:
        for t0 in range(0, vis.shape[1] - chunk + 1, chunk):
            piece = dev[:, t0:t0 + chunk].contiguous()
            p.search([piece.data_ptr()], torch.cuda.current_stream().cuda_stream)
            n = p.info()["n_windows"]
            if n:
                rows.append(p.windows(np.arange(n)))
            c = p.candidates()
            if len(c):
                cands.append(c)
            torch.cuda.synchronize()
    table = np.concatenate(rows) if rows else np.zeros(0)
    cands = np.concatenate(cands) if cands else np.zeros(0, table.dtype)
    return table, cands


@pytest.mark.parametrize("ws,chunks", [
    ([1, 2, 4, 8, 16, 32], [976, 244, 61, 1000, 7]),
    ([1, 4, 64], [300, 61]),
    ([1, 4, 64, 128], [300, 61]),
], ids=["fused", "fused-64", "two-pass"])
def test_stream_equals_batch(ws, chunks):
    spec = synth.evn_scan(4021, 3, 2928, 8, 32, 1.024e-3, 16e6, 3, width_max=32, n_tones=1)
    vis = spec.full()
    desc = spec.desc()
    thr = 4.5
    batch, bc = _batch(desc, vis, ws, thr)
    bmap = {_key(r): r for r in batch}
    for chunk in chunks:
        print(f"case: windows {ws}, chunk {chunk}", flush=True)
        n_used = (vis.shape[1] // chunk) * chunk
        table, cands = _streamed(desc, vis, ws, thr, chunk)
        keys = [_key(r) for r in table]
        assert len(keys) == len(set(keys)), "a window was reported twice"
        # exactly the batch windows that end within the APs streamed so far
        want = {k for k in bmap if k[3] + k[2] <= n_used}
        assert set(keys) == want
        for r in table:
            b = bmap[_key(r)]
            for f in ("k_rate", "k_delay", "amp", "snr", "energy", "delay_s", "rate_hz"):
                assert r[f] == b[f], (chunk, _key(r), f, r[f], b[f])
        ck = sorted(_key(c) for c in cands)
        assert ck == sorted(k for k in (_key(c) for c in bc) if k[3] + k[2] <= n_used)


def test_stream_against_reference():
    """A few chunks of a stream, each call's windows against the CPU reference."""
    spec = synth.evn_scan(4077, 3, 700, 8, 32, 1.024e-3, 16e6, 2, width_max=16)
    vis = spec.full()
    desc = spec.desc()
    ws, thr = [1, 2, 4, 8, 16, 32], 4.5
    table, _ = _streamed(desc, vis, ws, thr, 175)
    ref = oracle_table([vis], [desc], ws, 4, 2, thr)
    rmap = {_key(r): i for i, r in enumerate(ref)}
    order = np.array([rmap[_key(r)] for r in table])
    fv = vis.reshape(vis.shape[0], vis.shape[1], -1)
    compare_windows(table, ref[order], lambda s, b: fv[b], 4, 2, "stream")
    assert len(table) == len(ref)


def test_stream_skipped_subarray_and_ids():
    """A subarray with no chunk in a call keeps its state; window ids of the
    call resolve to their absolute starts."""
    import torch

    import paper_2108_05602_amd as F
    specs = [synth.evn_scan(4100 + i, 3, 400, 8, 32, 1.024e-3, 16e6, 1, width_max=8)
             for i in range(2)]
    vis = [s.full() for s in specs]
    ws, chunk = [1, 2, 4, 8], 100
    descs = [dict(s.desc(), n_ap=chunk) for s in specs]
    dev = [torch.from_numpy(v).cuda() for v in vis]
    st = torch.cuda.current_stream().cuda_stream
    got = {0: [], 1: []}
    with F.Plan(descs, ws, snr_threshold=4.5, flags=F.FRINGE_STREAMING) as p:
        # subarray 1 skips the second call, then catches up
        schedule = [(0, 0), (0, None), (1, 1), (2, 2), (3, 3)]
        for c0, c1 in schedule:
            ptrs = []
            for s, c in ((0, c0), (1, c1)):
                if c is None:
                    ptrs.append(None)
                else:
                    piece = dev[s][:, c * chunk:(c + 1) * chunk].contiguous()
                    ptrs.append(piece)
            p.search([t.data_ptr() if t is not None else None for t in ptrs], st)
            n = p.info()["n_windows"]
            rows = p.windows(np.arange(n)) if n else []
            for r in rows:
                got[int(r["scan"])].append(_key(r)[1:])
            for r in rows[:5]:
                assert p.window_id(int(r["scan"]), int(r["baseline"]), int(r["window_ap"]),
                                   int(r["t_start"])) == int(np.nonzero((rows["scan"] == r["scan"]) &
                                   (rows["baseline"] == r["baseline"]) & (rows["window_ap"] == r["window_ap"]) &
                                   (rows["t_start"] == r["t_start"]))[0][0])
            del ptrs
    # subarray 1: chunks 0,1,2,3 = the whole 400-AP scan: every window once
    batch1, _ = _batch(specs[1].desc(), vis[1], ws, 4.5)
    assert sorted(got[1]) == sorted(_key(r)[1:] for r in batch1)


def test_stream_alternating_streams():
    """Chunks of one streaming plan searched on two HIP streams in turn (each
    search waits for the previous one, whose stage it reads): streamed ==
    batch, bit for bit."""
    import torch

    import paper_2108_05602_amd as F
    spec = synth.evn_scan(4031, 3, 1952, 8, 32, 1.024e-3, 16e6, 3, width_max=32, n_tones=1)
    vis = spec.full()
    desc = spec.desc()
    ws, thr, chunk = [1, 2, 4, 8, 16, 32], 4.5, 244
    print(f"case: alternating streams, chunk {chunk}", flush=True)
    batch, _ = _batch(desc, vis, ws, thr)
    bmap = {_key(r): r for r in batch}
    dev = torch.from_numpy(vis).cuda()
    pieces = [dev[:, t0:t0 + chunk].contiguous() for t0 in range(0, vis.shape[1], chunk)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = []
    with F.Plan([dict(desc, n_ap=chunk)], ws, pad_freq=4, pad_time=2, snr_threshold=thr,
                flags=F.FRINGE_STREAMING) as p:
        for i, piece in enumerate(pieces):
            p.search([piece.data_ptr()], streams[i % 2].cuda_stream)
            n = p.info()["n_windows"]
            if n:
                got.append(p.windows(np.arange(n)))
    table = np.concatenate(got)
    assert {_key(r) for r in table} == set(bmap)
    for r in table:
        b = bmap[_key(r)]
        for f in ("k_rate", "k_delay", "amp", "snr", "energy"):
            assert r[f] == b[f], (_key(r), f)


@pytest.mark.parametrize("ws,chunk", [([1, 2, 4, 8, 16, 32], 244), ([1, 2, 4, 8, 16, 32], 7),
                                      ([1, 4, 64, 128], 61)],
                         ids=["fused", "short-chunk", "two-pass"])
def test_stream_reused_buffer(ws, chunk):
    """The chunk is read where the caller holds it: one device buffer serves
    every chunk, refilled on the search's stream right after each search is
    enqueued (no host synchronisation in between), and the records still
    equal the batch search's (the next call's halo is taken during the call)."""
    import torch

    import paper_2108_05602_amd as F
    spec = synth.evn_scan(4033, 3, 1464, 8, 32, 1.024e-3, 16e6, 2, width_max=32, n_tones=1)
    vis = spec.full()
    desc = spec.desc()
    thr = 4.5
    print(f"case: reused chunk buffer, windows {ws}, chunk {chunk}", flush=True)
    batch, _ = _batch(desc, vis, ws, thr)
    bmap = {_key(r): r for r in batch}
    dev = torch.from_numpy(vis).cuda()
    n_used = (vis.shape[1] // chunk) * chunk
    st = torch.cuda.current_stream()
    buf = dev[:, :chunk].clone().contiguous()
    got = []
    with F.Plan([dict(desc, n_ap=chunk)], ws, pad_freq=4, pad_time=2, snr_threshold=thr,
                flags=F.FRINGE_STREAMING) as p:
        for t0 in range(0, n_used, chunk):
            p.search([buf.data_ptr()], st.cuda_stream)
            nxt = t0 + chunk
            # stream-ordered after the search: the next chunk, or garbage
            if nxt < n_used:
                buf.copy_(dev[:, nxt:nxt + chunk])
            else:
                buf.fill_(float("nan"))
            n = p.info()["n_windows"]
            if n:
                got.append(p.windows(np.arange(n)))
    table = np.concatenate(got)
    keys = [_key(r) for r in table]
    assert len(keys) == len(set(keys))
    assert set(keys) == {k for k in bmap if k[3] + k[2] <= n_used}
    for r in table:
        b = bmap[_key(r)]
        for f in ("k_rate", "k_delay", "amp", "snr", "energy"):
            assert r[f] == b[f], (chunk, _key(r), f, r[f], b[f])
