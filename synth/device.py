"""Device-side generation of the synthetic scans, for workloads too large to
build in host memory (the batched uneven recipe is about 1.3 TB, more than
the GPU's HBM too, so it is generated and searched in waves).

Same recipe as the host generator (synth.ScanSpec): complex Gaussian noise
with N(0, 1) real and imaginary parts, plus the spec's pulses, tones and
bursts, with the same event parameters (drawn on the host by the spec's
constructor).  Only the noise stream differs: baseline b of a scan with seed
s draws its noise from torch's CUDA generator seeded with
noise_seed(s, b) (real and imaginary parts interleaved), so any baseline can
be regenerated alone, bit for bit, on the same device and software.  The
injected signals are computed in float64 and rounded to complex64, like the
host generator's.

This module makes input data only; it holds none of the search arithmetic.
Tests that compare a search of device-generated data with the CPU reference
copy the windows they check back to the host.
"""

from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from . import SIGMA_C, ScanSpec, baseline_pairs


def noise_seed(seed: int, b: int) -> int:
    """Seed of baseline b's noise stream in a scan of the given seed."""
    return (int(seed) * 1_000_003 + 1 + int(b)) & ((1 << 63) - 1)


def fill(spec: ScanSpec, out, b_lo: int = 0) -> None:
    """Write baselines [b_lo, b_lo + out.shape[0]) of the scan into `out`, a
    complex64 CUDA tensor of shape (nb, n_ap, n_if, n_chan) or (nb, n_ap, F)."""
    import torch

    nb = out.shape[0]
    big_f = spec.n_freq
    x = out.reshape(nb, spec.n_ap, big_f)
    dev = out.device
    for k in range(nb):
        b = b_lo + k
        if spec.noise:
            g = torch.Generator(device=dev)
            g.manual_seed(noise_seed(spec.seed, b))
            torch.view_as_real(x[k]).normal_(0.0, 1.0, generator=g)
        else:
            x[k].zero_()
    pairs = baseline_pairs(spec.n_stations) if spec.n_stations > 1 else [(0, 0)]
    pairs = pairs + [(0, 0)] * max(0, b_lo + nb - len(pairs))
    ii = np.array([pairs[b][0] for b in range(b_lo, b_lo + nb)])
    jj = np.array([pairs[b][1] for b in range(b_lo, b_lo + nb)])
    f_hz = torch.arange(big_f, dtype=torch.float64, device=dev) * spec.chan_width_hz
    for p in spec.pulses:
        t0, t1 = p.start, min(spec.n_ap, p.start + p.width)
        if t1 <= t0:
            continue
        sel = np.arange(nb) if p.baselines is None else np.array(
            [k for k in range(nb) if (b_lo + k) in p.baselines], dtype=np.int64)
        if sel.size == 0:
            continue

        def diff(v):
            v = np.asarray(v, dtype=np.float64)
            return v[ii[sel]] - v[jj[sel]] if v.size > 1 else np.full(sel.size, float(v[0]))

        tau = torch.from_numpy(diff(p.tau_s)).to(dev)
        nu = torch.from_numpy(diff(p.nu_s)).to(dev)
        phi = torch.from_numpy(diff(p.phi_s)).to(dev)
        a = p.amp if p.amp is not None else p.snr * SIGMA_C / math.sqrt(p.width * big_f)
        t_s = torch.arange(t0, t1, dtype=torch.float64, device=dev) * spec.ap_seconds
        ph = 2.0 * math.pi * (f_hz[None, None, :] * tau[:, None, None] +
                              t_s[None, :, None] * nu[:, None, None]) + phi[:, None, None]
        sig = (a * torch.exp(1j * ph)).to(torch.complex64)
        idx = torch.from_numpy(sel).to(dev)
        x[idx, t0:t1] += sig
    for r in spec.tones:
        k = r.baseline - b_lo
        if not 0 <= k < nb:
            continue
        t0, t1 = r.start, min(spec.n_ap, r.start + r.length)
        t_s = torch.arange(t0, t1, dtype=torch.float64, device=dev) * spec.ap_seconds
        x[k, t0:t1, r.chan] += (r.amp * torch.exp(1j * (2 * math.pi * r.rate_hz * t_s + r.phase))
                                ).to(torch.complex64)
    for r in spec.bursts:
        k = r.baseline - b_lo
        if not 0 <= k < nb:
            continue
        t0, t1 = r.start, min(spec.n_ap, r.start + r.length)
        x[k, t0:t1, :] += complex(np.complex64(r.amp * np.exp(1j * r.phase)))


def generate(spec: ScanSpec, device="cuda:0"):
    """The whole scan as a complex64 tensor (B, n_ap, n_if, n_chan) on `device`."""
    import torch

    out = torch.empty((spec.n_baselines, spec.n_ap, spec.n_if, spec.n_chan),
                      dtype=torch.complex64, device=device)
    fill(spec, out)
    return out


def waves(specs: Sequence[ScanSpec], wave_bytes: int) -> List[List[int]]:
    """Scan indices packed in order into waves of at most wave_bytes of
    visibilities each (a scan larger than that is a wave of its own)."""
    out, cur, used = [], [], 0
    for i, s in enumerate(specs):
        n = s.nbytes()
        if cur and used + n > wave_bytes:
            out.append(cur)
            cur, used = [], 0
        cur.append(i)
        used += n
    if cur:
        out.append(cur)
    return out
