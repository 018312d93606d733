"""Every grid bin of every window against the direct DFT of the CPU reference
(P7), and Parseval on the GPU's own grid (P2), for the rate-transform forms
the 64-AP workload does not reach: the run-time sub-transform loop of long
windows (W = 64 at pad_time 2, eight sub-transforms), the LDS-ring kernel of
128-AP windows (pad_time 2 and 1), and M_f = 4096 (a band of 1,024 channels,
searched in spectra mode)."""

import numpy as np
import pytest

import oracle.fringe_oracle as fo
from fringe_testlib import run_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # (n_ap, n_if, n_chan, windows, pad_f, pad_t)
    (100, 2, 16, [64], 4, 2),        # S = 8 run-time loop
    (200, 2, 32, [128], 4, 2),       # LDS ring kernel, 16 sub-transforms
    (330, 1, 64, [2, 128], 2, 1),    # LDS ring kernel at pad_time 1, with short windows
    (12, 16, 64, [1, 4], 4, 2),      # M_f = 4096, spectra mode
]


@pytest.mark.parametrize("case", CASES, ids=[f"g{i}" for i in range(len(CASES))])
def test_grid_bins_and_parseval(case):
    import paper_2108_05602_amd as F
    t, n_if, n_chan, ws, pf, pt = case
    print(f"case: grid dump {case}", flush=True)
    rng = np.random.default_rng([91, t, n_chan])
    f = n_if * n_chan
    v = (rng.standard_normal((1, t, n_if, n_chan)) +
         1j * rng.standard_normal((1, t, n_if, n_chan))).astype(np.complex64)
    d = dict(n_baselines=1, n_ap=t, n_if=n_if, n_chan=n_chan, ap_seconds=1e-3,
             chan_width_hz=1e6)
    plan, table, _ = run_gpu([d], [v], ws, pf, pt, 50.0, flags=F.FRINGE_DUMP_GRID)
    x = v.reshape(t, f)
    y = fo.delay_spectra(x, pf)
    m_f = pf * f
    for i, row in enumerate(table):
        w, t0 = int(row["window_ap"]), int(row["t_start"])
        m_t = pt * w
        g = plan.grid(i, m_t, m_f)
        ref = fo.window_grid(y, t0, w, pt)
        scale = np.abs(ref).max()
        assert np.allclose(g, ref, rtol=0, atol=3e-6 * scale), (case, w, t0)
        e = float(np.sum(np.abs(x[t0:t0 + w]).astype(np.float64) ** 2))
        assert float(np.sum(np.abs(g.astype(np.complex128)) ** 2)) == \
            pytest.approx(m_t * m_f * e, rel=2e-5), (case, w, t0)
    plan.close()
