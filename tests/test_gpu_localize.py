"""Search, match and localize, end to end: three pulses from a source offset
by (3, -2) micro-radians from its a priori position, seen by ten stations
(Earth-fixed positions over a European-sized array) whose residual delays
are the geometric delays of the offset, are found by the GPU search, matched
into single pulses, and localized by Eq. (2) from their baseline delays.
The delays come quantised to the delay bins (1.95 ns), which bounds the
solution's error (about 2e-8 rad on this geometry); the check allows 6e-8.
"""

import numpy as np
import pytest

import oracle.pulse_match_oracle as pm
import synth

pytestmark = pytest.mark.gpu

RA0, DEC0, GAST = 1.0, 0.6, 2.0
OFFSET = np.array([3e-6, -2e-6])


def _stations(n=10, seed=8):
    rng = np.random.default_rng(seed)
    r = 6.371e6
    lat = np.radians(rng.uniform(40, 60, n))
    lon = np.radians(rng.uniform(-10, 30, n))
    return np.stack([r * np.cos(lat) * np.cos(lon), r * np.cos(lat) * np.sin(lon),
                     r * np.sin(lat)], 1)


def _s_hat(ra, dec):
    h = GAST - ra
    return np.array([np.cos(dec) * np.cos(h), -np.cos(dec) * np.sin(h), np.sin(dec)])


def test_search_match_localize():
    import torch

    import paper_2108_05602_amd as F
    st = _stations()
    # residual station delays: the offset source's geometric delay minus the a priori one
    tau_s = -(st @ (_s_hat(RA0 + OFFSET[0], DEC0 + OFFSET[1]) - _s_hat(RA0, DEC0))) / pm.C_LIGHT
    spec = synth.ScanSpec(seed=31, n_stations=10, n_ap=3000, n_if=8, n_chan=32,
                          ap_seconds=1.024e-3, chan_width_hz=0.5e6)
    rng = np.random.default_rng(3)
    for start in (500, 1500, 2500):
        spec.pulses.append(synth.Pulse(start=start, width=8, snr=20.0, tau_s=tau_s,
                                       nu_s=np.zeros(10), phi_s=rng.uniform(0, 2 * np.pi, 10)))
    print("case: search, match, localize; 10 stations x 3000 AP", flush=True)
    v = spec.full(threads=8)
    dev = torch.from_numpy(v).to("cuda:0")
    p = synth.C2_PARAMS
    with F.Plan([spec.desc()], p["window_aps"], pad_freq=p["pad_freq"], pad_time=p["pad_time"],
                snr_threshold=p["snr_threshold"]) as plan:
        plan.search([dev.data_ptr()], torch.cuda.current_stream().cuda_stream)
        cands = plan.candidates()
    rows, n_p = F.fringe_match(cands, 2, 5)
    assert n_p == 3
    pairs = synth.baseline_pairs(10)
    for pid in range(n_p):
        sel = rows[rows["pulse"] == pid]
        assert len(sel) >= 40                     # nearly every one of the 45 baselines
        b_xyz = np.array([st[pairs[b][0]] - st[pairs[b][1]] for b in sel["baseline"]])
        da, dd = F.fringe_delay_partials(b_xyz, GAST, RA0, DEC0)
        sol, rms, loo, loo_rms = F.fringe_localize(sel["delay_s"], da, dd)
        assert np.all(np.abs(sol - OFFSET) < 6e-8), (pid, sol)
        assert rms < 1.5e-9
        assert np.all(np.abs(loo - OFFSET) < 1e-7)
        ref = pm.localize(sel["delay_s"], *pm.delay_partials(b_xyz, GAST, RA0, DEC0))
        np.testing.assert_allclose(sol, ref[0], rtol=1e-9)
