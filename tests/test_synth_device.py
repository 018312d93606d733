"""The device-side generator (synth.device) on CPU tensors: the injected
signals equal the host generator's, the noise has the recipe's statistics
and regenerates bit for bit per baseline, and waves pack scans in order
within their byte budget."""

import numpy as np
import pytest
import torch

import synth
from synth import device as sd


def _small_spec(noise):
    s = synth.evn_scan(77, 5, 400, 4, 16, 1.024e-3, 16e6, 4, width_max=32, n_tones=3,
                       n_bursts=3, burst_len=(1, 40), noise=noise)
    s.pulses[1].baselines = [0, 3, 7]
    return s


def test_signals_match_host_generator():
    spec = _small_spec(noise=False)
    host = spec.full(threads=1)
    dev = torch.empty(host.shape, dtype=torch.complex64)
    sd.fill(spec, dev)
    got = dev.numpy()
    assert np.abs(got).max() > 0.1
    assert np.allclose(got, host, rtol=0, atol=2e-6 * np.abs(host).max())
    # a slab of baselines alone gives the same rows
    part = torch.empty((4,) + host.shape[1:], dtype=torch.complex64)
    sd.fill(spec, part, b_lo=3)
    assert np.array_equal(part.numpy(), got[3:7])


def test_noise_statistics_and_regeneration():
    spec = _small_spec(noise=True)
    spec.pulses.clear()
    spec.tones.clear()
    spec.bursts.clear()
    a = torch.empty((spec.n_baselines, spec.n_ap, spec.n_if, spec.n_chan), dtype=torch.complex64)
    sd.fill(spec, a)
    r = torch.view_as_real(a).numpy().astype(np.float64)
    assert abs(r.mean()) < 0.01
    assert r[..., 0].var() == pytest.approx(1.0, abs=0.02)
    assert r[..., 1].var() == pytest.approx(1.0, abs=0.02)
    assert abs(np.corrcoef(r[..., 0].ravel(), r[..., 1].ravel())[0, 1]) < 0.01
    one = torch.empty((1,) + tuple(a.shape[1:]), dtype=torch.complex64)
    sd.fill(spec, one, b_lo=6)
    assert torch.equal(one[0], a[6])
    assert not torch.equal(a[5], a[6])
    assert sd.noise_seed(3000, 1) != sd.noise_seed(3001, 0)


def test_waves_pack_in_order():
    specs = synth.c3(n_scans=30)
    budget = 40_000_000_000
    w = sd.waves(specs, budget)
    assert [i for g in w for i in g] == list(range(30))
    for g in w:
        size = sum(specs[i].nbytes() for i in g)
        assert size <= budget or len(g) == 1
    for a, b in zip(w, w[1:]):
        assert sum(specs[i].nbytes() for i in a) + specs[b[0]].nbytes() > budget
