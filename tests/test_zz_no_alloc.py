"""The allocation-free search (fringe_search_noalloc) through the C ABI on
cuda:0, against the planned search (fringe_plan + fringe_search +
candidates_get) on the same inputs: two calls in a row, the second on a
smaller scan (the static scratch keeps the first call's contents), then a
delay-only call; candidate keys and bins exact, amp, SNR and energy within
the 1e-4 parity tolerance.  Plus the host-side refusals: a scan whose work
buffers exceed the scratch, unsupported flags, windows longer than 64 APs."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-4


def _planned(desc, ws, dev, flags=0, thr=4.5):
    import torch

    import paper_2108_05602_amd as F
    with F.Plan([desc], ws, pad_freq=4, pad_time=2, snr_threshold=thr, max_candidates=1 << 20,
                flags=flags) as p:
        p.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        return p.candidates()


def _noalloc(desc, ws, dev, capacity, flags=0, thr=4.5):
    import torch

    from paper_2108_05602_amd import binding as B
    out = torch.zeros(capacity * B.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream()
    B.fringe_search_noalloc(desc, ws, dev.data_ptr(), out.data_ptr(), capacity, total.data_ptr(),
                            pad_freq=4, pad_time=2, snr_threshold=thr, flags=flags,
                            stream=st.cuda_stream)
    torch.cuda.synchronize()
    n = int(total.item())
    recs = np.frombuffer(out.cpu().numpy().tobytes(), dtype=B.CANDIDATE_DTYPE)[:min(n, capacity)]
    return n, recs


def _same(a, b, label):
    assert len(a) == len(b), (label, len(a), len(b))
    for k in ("scan", "baseline", "window_ap", "t_start", "k_rate", "k_delay"):
        assert np.array_equal(a[k], b[k]), (label, k)
    for k in ("amp", "snr", "energy"):
        assert np.allclose(a[k], b[k], rtol=RTOL, atol=1e-6), (label, k)


def test_noalloc_equals_planned_search():
    import torch
    print("case: no-alloc search vs planned search, two calls in a row", flush=True)
    ws = [1, 2, 4, 8, 16, 32]
    big = synth.evn_scan(4201, 6, 976, 8, 32, 1.024e-3, 16e6, 3, width_max=32, n_tones=1)
    small = synth.evn_scan(4202, 3, 333, 8, 32, 1.024e-3, 16e6, 2, width_max=16)
    for label, spec, cap in (("first, 15 BL x 976 AP", big, 1 << 14),
                             ("second, 3 BL x 333 AP", small, 1 << 14)):
        dev = torch.from_numpy(spec.full()).cuda()
        want = _planned(spec.desc(), ws, dev)
        n, got = _noalloc(spec.desc(), ws, dev, cap)
        assert n == len(want), (label, n, len(want))
        _same(got, want, label)
        print(f"{label}: {n} candidates equal", flush=True)
    # a capacity below the total keeps the first records in key order
    dev = torch.from_numpy(big.full()).cuda()
    want = _planned(big.desc(), ws, dev)
    n, got = _noalloc(big.desc(), ws, dev, 5)
    assert n == len(want) and len(got) == 5
    _same(got, want[:5], "capacity 5")
    # delay-only search
    want = _planned(small.desc(), ws, torch.from_numpy(small.full()).cuda(),
                    flags=0x20, thr=4.0)
    n, got = _noalloc(small.desc(), ws, torch.from_numpy(small.full()).cuda(), 1 << 14,
                      flags=0x20, thr=4.0)
    assert n == len(want)
    _same(got, want, "delay-only")


def test_noalloc_refusals():
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd import binding as B
    dev = torch.zeros(8, dtype=torch.complex64, device="cuda")
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    huge = dict(n_baselines=45, n_ap=58600, n_if=8, n_chan=32, ap_seconds=1e-3, chan_width_hz=5e5)
    with pytest.raises(F.FringeError) as e:
        B.fringe_search_noalloc(huge, [1, 2, 4], dev.data_ptr(), out.data_ptr(), 1, tot.data_ptr())
    assert e.value.code == B.FRINGE_E_NOMEM and "static scratch" in str(e.value)
    ok = dict(n_baselines=1, n_ap=64, n_if=2, n_chan=16, ap_seconds=1.0, chan_width_hz=1.0)
    with pytest.raises(F.FringeError) as e:
        B.fringe_search_noalloc(ok, [4], dev.data_ptr(), out.data_ptr(), 1, tot.data_ptr(),
                                flags=B.FRINGE_STREAMING)
    assert e.value.code == B.FRINGE_E_INVALID
    with pytest.raises(F.FringeError) as e:
        B.fringe_search_noalloc(dict(ok, n_ap=300), [128], dev.data_ptr(), out.data_ptr(), 1,
                                tot.data_ptr())
    assert e.value.code == B.FRINGE_E_UNSUPPORTED
