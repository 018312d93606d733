"""The time chunk of a plan (fringe_plan_set_chunk) on cuda:0.

  * every chunk (64, 256, 1024 APs and the automatic one) gives the same
    records, bit for bit, in batch plans and in streaming plans with and
    without dedispersion shifts (shifts and chunk set in either order);
  * the argument rules: a chunk off the search period or outside
    [64, 1024], a scan out of range, after the first search, a plan with
    windows longer than 64 APs;
  * a server whose plans take a longer chunk returns every chunk's
    candidates unchanged, and a server with dedispersion shifts returns
    those of a streaming plan with the same shifts.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WS = [1, 2, 4, 8, 16, 32]
FIELDS = ("scan", "baseline", "window_ap", "t_start", "k_rate", "k_delay", "amp", "snr", "energy")


def _all(plan):
    n = plan.info()["n_windows"]
    return plan.windows(np.arange(n, dtype=np.int64))


def _same(a, b, label):
    assert len(a) == len(b), label
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (label, f)


def _shifts(desc, dm):
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    f = channel_freqs_hz(1.6e9, desc["n_if"], desc["n_chan"], desc["chan_width_hz"])
    return dm_shifts(dm, f, desc["ap_seconds"])


def test_chunk_gives_identical_records():
    import torch

    import paper_2108_05602_amd as F
    print("case: batch plan, chunks auto / 64 / 256 / 1024", flush=True)
    spec = synth.evn_scan(4601, 4, 2300, 8, 32, 1.024e-3, 16e6, 3, width_max=32, n_tones=1)
    desc = spec.desc()
    dev = torch.from_numpy(spec.full()).cuda()
    st = torch.cuda.current_stream().cuda_stream
    with F.Plan([desc], WS, snr_threshold=4.5) as p:
        auto = p.chunk(0)
        p.search([dev.data_ptr()], st)
        ref, ref_c = _all(p), p.candidates()
    assert auto in (64, 128, 256, 512, 1024)
    for c in (64, 256, 1024):
        with F.Plan([desc], WS, snr_threshold=4.5) as p:
            p.set_chunk(0, c)
            assert p.chunk(0) == c
            p.search([dev.data_ptr()], st)
            _same(_all(p), ref, f"chunk {c}")
            _same(p.candidates(), ref_c, f"chunk {c} candidates")
    with F.Plan([desc], WS, snr_threshold=4.5) as p:
        p.set_chunk(0, 512)
        p.set_chunk(0, 0)
        assert p.chunk(0) == auto


def test_chunk_rules():
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd import binding as B
    print("case: set_chunk argument rules", flush=True)
    spec = synth.evn_scan(4602, 3, 400, 8, 32, 1.024e-3, 16e6, 1, width_max=8)
    desc = spec.desc()
    dev = torch.from_numpy(spec.full()).cuda()
    with F.Plan([desc], WS, snr_threshold=4.5) as p:
        for bad in (100, 32, 2048, -64):
            with pytest.raises(F.FringeError) as e:
                p.set_chunk(0, bad)
            assert e.value.code == B.FRINGE_E_INVALID
        with pytest.raises(F.FringeError) as e:
            p.set_chunk(1, 256)
        assert e.value.code == B.FRINGE_E_INVALID
        p.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        p.candidates()
        with pytest.raises(F.FringeError) as e:
            p.set_chunk(0, 256)
        assert e.value.code == B.FRINGE_E_STATE
    with F.Plan([desc], WS + [64, 128], snr_threshold=4.5) as p:
        with pytest.raises(F.FringeError) as e:
            p.set_chunk(0, 256)
        assert e.value.code == B.FRINGE_E_UNSUPPORTED


@pytest.mark.parametrize("order", ["shifts-first", "chunk-first"])
def test_streaming_chunk_with_shifts(order):
    import torch

    import paper_2108_05602_amd as F
    print(f"case: streaming plan, shifts and chunk 512 ({order})", flush=True)
    spec = synth.evn_scan(4603, 3, 5 * 488, 8, 32, 1.024e-3, 16e6, 3, width_max=32, n_tones=1)
    desc = dict(spec.desc(), n_ap=488)
    vis = torch.from_numpy(spec.full()).cuda()
    pieces = [vis[:, k * 488:(k + 1) * 488].contiguous() for k in range(5)]
    sh = torch.from_numpy(_shifts(desc, 200.0)).cuda()
    st = torch.cuda.current_stream().cuda_stream

    def run(chunk):
        out = []
        with F.Plan([desc], WS, snr_threshold=4.5, flags=F.FRINGE_STREAMING) as p:
            if order == "chunk-first" and chunk:
                p.set_chunk(0, chunk)
            p.set_shifts(0, sh.data_ptr())
            if order == "shifts-first" and chunk:
                p.set_chunk(0, chunk)
            if chunk:
                assert p.chunk(0) == chunk
            for piece in pieces:
                p.search([piece.data_ptr()], st)
                out.append(_all(p))
        return out

    ref, got = run(0), run(512)
    assert sum(len(r) for r in ref) > 0
    for k, (a, b) in enumerate(zip(got, ref)):
        _same(a, b, f"call {k}")


def test_server_chunk_and_shifts():
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.serve import FringeServer, run_schedule
    print("case: server with time_chunk 256, and with dedispersion shifts", flush=True)
    chunk, n_chunks = 488, 4
    specs = [synth.evn_scan(4610 + i, n_st, chunk * n_chunks, 8, 32, 1.024e-3, 16e6, 2,
                            width_max=16, n_tones=1) for i, n_st in enumerate([3, 5])]
    vis = [torch.from_numpy(s.full()).cuda() for s in specs]
    payloads = [[v[:, k * chunk:(k + 1) * chunk].contiguous() for k in range(n_chunks)] for v in vis]
    subs = [dict(s.desc(), n_ap=chunk) for s in specs]
    sched = [(0.0, s, k) for s in range(2) for k in range(n_chunks)]

    def serve(**kw):
        srv = FringeServer(subs, WS, snr_threshold=4.5, **kw)
        try:
            res = run_schedule(srv, sched, payloads).results
        finally:
            srv.close()
        return {(r.sub, r.seq): r.candidates for r in res}

    base, longer = serve(), serve(time_chunk=256)
    assert set(base) == set(longer)
    for k in base:
        _same(longer[k], base[k], f"server chunk {k}")
    sh = [torch.from_numpy(_shifts(sd, 150.0)).cuda() for sd in subs]
    ded = serve(shifts=sh)
    st = torch.cuda.current_stream().cuda_stream
    for s in range(2):
        with F.Plan([subs[s]], WS, snr_threshold=4.5, flags=F.FRINGE_STREAMING) as p:
            p.set_shifts(0, sh[s].data_ptr())
            for k in range(n_chunks):
                p.search([payloads[s][k].data_ptr()], st)
                _same(ded[(s, k)], p.candidates(), f"dedispersed server {s}/{k}")
