"""Dedispersion in streaming plans on cuda:0: a subarray's scan fed chunk by
chunk, with shifts up to D APs set before the first search, gives exactly
the windows of a batch search (with the same shifts) of the concatenated
APs that end at least D APs before the end of the data received, with
bit-identical records, for chunks longer and shorter than D; in the full
and the delay-only search.  Shifts are refused once the plan has searched."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _key(r):
    return (int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))


def _shifts(desc, dm):
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    f = channel_freqs_hz(1.6e9, desc["n_if"], desc["n_chan"], desc["chan_width_hz"])
    return dm_shifts(dm, f, desc["ap_seconds"])


@pytest.mark.parametrize("flags", [0, 0x20], ids=["full", "delay-only"])
def test_streamed_dedispersion_equals_batch(flags):
    import torch

    import paper_2108_05602_amd as F
    spec = synth.evn_scan(4431, 3, 2440, 8, 32, 1.024e-3, 16e6, 4, width_max=32, n_tones=1)
    vis = spec.full()
    desc = spec.desc()
    sh = _shifts(desc, 300.0)
    d_max = int(sh.max())
    assert d_max > 61
    ws, thr = [1, 2, 4, 8, 16, 32], 4.5
    dev = torch.from_numpy(vis).cuda()
    sh_dev = torch.from_numpy(sh).cuda()
    st = torch.cuda.current_stream().cuda_stream
    with F.Plan([desc], ws, pad_freq=4, pad_time=2, snr_threshold=thr, flags=flags) as bp:
        bp.set_shifts(0, sh_dev.data_ptr())
        bp.search([dev.data_ptr()], st)
        batch = bp.windows(np.arange(bp.info()["n_windows"]))
    bmap = {_key(r): r for r in batch}
    for chunk in (976, 300, 61):
        print(f"case: streamed dedispersion, flags {flags}, chunk {chunk}, D = {d_max}", flush=True)
        pieces = [dev[:, t0:t0 + chunk].contiguous() for t0 in range(0, vis.shape[1] - chunk + 1, chunk)]
        n_used = len(pieces) * chunk
        rows = []
        with F.Plan([dict(desc, n_ap=chunk)], ws, pad_freq=4, pad_time=2, snr_threshold=thr,
                    flags=F.FRINGE_STREAMING | flags) as p:
            p.set_shifts(0, sh_dev.data_ptr())
            for piece in pieces:
                p.search([piece.data_ptr()], st)
                n = p.info()["n_windows"]
                if n:
                    rows.append(p.windows(np.arange(n)))
            with pytest.raises(F.FringeError):
                p.set_shifts(0, sh_dev.data_ptr())
        table = np.concatenate(rows)
        keys = [_key(r) for r in table]
        assert len(keys) == len(set(keys))
        want = {k for k in bmap if k[2] + k[1] <= n_used - d_max}
        assert set(keys) == want
        for r in table:
            b = bmap[_key(r)]
            for f in ("k_rate", "k_delay", "amp", "snr", "energy"):
                assert r[f] == b[f], (chunk, _key(r), f)
