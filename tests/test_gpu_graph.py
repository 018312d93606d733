"""FRINGE_GRAPH on cuda:0: a batch search captured in a HIP graph and replayed.

Every replay, with the program's own eager work and synchronizations in
between, gives the eager search's window table and candidate list bit for
bit; a new input is captured anew and again matches the eager search.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _tables(plan):
    n = plan.info()["n_windows"]
    return plan.windows(np.arange(n)), plan.candidates()


def _same(a, b, what):
    assert len(a) == len(b), what
    for k in a.dtype.names:
        assert np.array_equal(a[k], b[k]), (what, k)


def test_graph_replays_equal_eager():
    import torch

    import paper_2108_05602_amd as F
    p = synth.C2_PARAMS
    specs = [synth.c2(seed=31 + i, n_stations=4, n_ap=1500, n_pulses=4, n_tones=1) for i in range(2)]
    vis = [torch.from_numpy(s.full()).cuda() for s in specs]
    desc = specs[0].desc()
    kw = dict(pad_freq=p["pad_freq"], pad_time=p["pad_time"], snr_threshold=p["snr_threshold"])
    st = torch.cuda.current_stream()
    want = []
    with F.Plan([desc], p["window_aps"], **kw) as eager:
        for v in vis:
            eager.search([v.data_ptr()], st.cuda_stream)
            want.append(_tables(eager))
    assert len(want[0][1]) > 0
    with F.Plan([desc], p["window_aps"], flags=F.FRINGE_GRAPH, **kw) as g:
        for rep, idx in enumerate([0, 0, 0, 1, 1, 0]):
            print(f"case: graph search {rep}, input {idx}", flush=True)
            g.search([vis[idx].data_ptr()], st.cuda_stream)
            t, c = _tables(g)
            _same(t, want[idx][0], f"table {rep}")
            _same(c, want[idx][1], f"candidates {rep}")
            x = torch.randn(1 << 20, device="cuda")
            assert float((x * 2).sum().item()) == float((x * 2).sum().item())
            torch.cuda.synchronize()
