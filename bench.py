#!/usr/bin/env python3
"""Fringe-search benchmark on one MI355X.

Headline workload: the batched uneven set of 200 scans (10-120 s of
1.024 ms APs, 3-12 stations = 3-66 baselines, 8 or 16 IF x 16/32/64
channels of 16 MHz IFs, pulses one per 3 s and narrowband RFI tones one per
6 s), windows of 1-64 APs at 50 % overlap, 4x delay / 2x rate padding,
threshold 4.5: about 1.1 G windows over 1.3 TB of visibilities, more than
the GPU holds.  The scans are generated on the device in waves of at most
--wave-gb of visibilities; each wave is one plan (one fused launch per fold
class of its bands), searched W times untimed and then K times timed.  A
step is one search of every wave (plus each search's candidate copy to the
host): ms_per_step is the sum over the waves of their timed search, each
bracketed by device synchronisations, averaged over the K steps; the
generation of a wave is outside every timed region, its data already in HBM
when each of its searches starts.

Further keys: the EVN-like single scan (45 baselines x 58,600 APs x 256
channels, windows 1-32 APs) with its calibrated, delay-only, DM-search,
plain-path, graph and serving legs; the large dense scan (66 baselines x
117,200 APs x 1,024 channels, windows 1-128 APs, 63.4 GB, generated on the
device); roof probes; the CPU reference on a bounded sample of the
headline workload.  Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--only c3|c2]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector, published
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E, published

# HBM bytes of one fused-kernel launch on the full EVN-like scan, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what
# the same counter read for a 1 GiB device copy (FETCH_SIZE x 1.99992,
# WRITE_SIZE x 1.0).  Valid only for the kernel and launch code they were
# taken on: `traffic` is reported as null when the hash of those sources
# (KERNEL_SOURCES) differs.
MEASURED_TRAFFIC = {
    "kernel_sha256": "7628d6b393b81f70bca09f0985786516a4f2f3b139266c821a33a7b0d0d9bafc",
    "fetch_bytes": 8398317766,
    "write_bytes": 2042506361,
}

# The fused search kernel of the EVN-like scan and the host code that sizes
# and launches it.
KERNEL_SOURCES = ("dev_common.h", "window_key.h", "fused_search.h", "kernels.h",
                  "fused_p2_w32.hip", "fused_dispatch.hip", "fringe_api.hip")

# HBM bytes of the batched headline's search kernels in one step (every
# launch of the fused kernel, in both modes, and of the delay transform),
# from the same counters and copy scaling (FETCH_SIZE x 1.99992,
# WRITE_SIZE x 1.0), with the launch configuration the autotuner chose then
# (per band: spectra mode, time chunk).  Reported only while the sources
# below hash alike and the run's tuning and launch count are the same.
MEASURED_TRAFFIC_C3 = {
    "kernel_sha256": "4b90d7d0c7392d72445054985f44d5a3d73224a89b2b5e4e6a98daebda43cbcf",
    "fused_fetch_bytes": 4959186448060,
    "fused_write_bytes": 321859739360,
    "delay_fetch_bytes": 1013316601416,
    "delay_write_bytes": 4058853977600,
    "fused_launches_per_step": 620,
    "delay_launches_per_step": 610,
    "tuning": {128: (1, 512), 256: (0, 512), 512: (1, 512), 1024: (1, 512)},
}


# The tune table the library's autotuner (FRINGE_AUTOTUNE) wrote on an
# MI355X for the headline's four classes of scans; plans look their classes
# up in it, and a device of another kind or size tunes them afresh.
SHIPPED_TUNE = os.path.join(ROOT, "paper_2108_05602_amd", "tune", "gfx950_256cu.json")

C3_SOURCES = ("csrc/dev_common.h", "csrc/window_key.h", "csrc/fused_search.h", "csrc/kernels.h",
              "csrc/fused_p2_w64.hip", "csrc/fused_x_p2.hip", "csrc/delay_fft.hip",
              "csrc/fused_dispatch.hip", "csrc/fringe_api.hip", "csrc/tune_table.cpp",
              "csrc/twiddles.hip", "../synth/__init__.py", "../synth/device.py")


def kernel_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for name in sources or KERNEL_SOURCES:
        h.update(name.encode())
        path = os.path.join(ROOT, "paper_2108_05602_amd", name if sources else os.path.join("csrc", name))
        with open(os.path.normpath(path), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def window_levels(n_ap, window_aps):
    out = []
    for w in window_aps:
        s = max(1, w // 2)
        out.append((w, s, (n_ap - w) // s + 1 if n_ap >= w else 0))
    return out


def algorithmic_flops(n_bl, n_ap, n_freq, window_aps, pad_f, pad_t):
    """Radix-2 operation counts: 5 N log2 N per N-point complex FFT, 5 per
    grid point for |G|^2, the max and the energy.  Returns (delay, rate,
    peak) flops of one full search."""
    m_f = pad_f * n_freq
    delay = n_bl * n_ap * 5.0 * m_f * math.log2(m_f)
    rate = peak = 0.0
    for w, s, n in window_levels(n_ap, window_aps):
        m_t = pad_t * w
        rate += n_bl * n * m_f * 5.0 * m_t * max(1.0, math.log2(m_t))
        peak += n_bl * n * m_f * m_t * 5.0
    return delay, rate, peak


def cpu_baseline(spec, params, n_bl=24, n_ap=4096, n_bl_one=1):
    """The CPU reference, as it stands, on a bounded sample of the same scan:
    with numpy's BLAS pool (the reported value) and on one thread, plus the
    projection of the full scan at the pool's rate."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import fringe_oracle as fo

    def run(n_b):
        xs = [spec.baseline(b, 0, n_ap).reshape(n_ap, -1) for b in range(n_b)]
        t0 = time.perf_counter()
        n = 0
        for b, x in enumerate(xs):
            n += len(fo.search_baseline(x, params["window_aps"], params["pad_freq"],
                                        params["pad_time"], spec.ap_seconds, spec.chan_width_hz,
                                        baseline=b))
        return n, time.perf_counter() - t0

    n, dt = run(n_bl)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        n1, dt1 = run(n_bl_one)
    n_full = sum(n_w for _, _, n_w in window_levels(spec.n_ap, params["window_aps"])) * spec.n_baselines
    return {"value": n / dt, "unit": "windows/s", "cores": int(threads), "kind": "oracle",
            "sample": f"baselines 0-{n_bl - 1} x APs 0-{n_ap - 1} of the same scan, all "
                      f"{len(params['window_aps'])} window lengths: {n} windows in {dt:.1f} s",
            "one_thread": {"value": n1 / dt1, "sample": f"baseline 0 x APs 0-{n_ap - 1}: "
                                                        f"{n1} windows in {dt1:.1f} s"},
            "full_scan_projection_s": n_full / (n / dt)}


def roof_probes(reps=5):
    """Achievable roofs of this device, by the library's probe kernels: an
    FP32 FMA loop (non-packed instructions, like the search) and a 1 GiB
    HBM copy; best of `reps` launches, timed with HIP events on the stream
    they run on."""
    import torch

    from paper_2108_05602_amd import binding as B
    st = torch.cuda.current_stream()
    n_blocks, iters = 256 * 16, 16384
    out = torch.empty(n_blocks * 256, dtype=torch.float32, device="cuda:0")
    best_fma = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fl = B.fringe_probe_fma(n_blocks, iters, out.data_ptr(), st.cuda_stream)
        e1.record(st)
        e1.synchronize()
        best_fma = max(best_fma, fl / (e0.elapsed_time(e1) / 1e3) / 1e12)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    best_copy = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        B.fringe_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, st.cuda_stream)
        e1.record(st)
        e1.synchronize()
        best_copy = max(best_copy, 2 * nbytes / (e0.elapsed_time(e1) / 1e3) / 1e9)
    assert torch.equal(src[:1024], dst[:1024]) and torch.isfinite(out).all()
    del src, dst, out
    return {"fp32_fma_tflops": best_fma, "hbm_copy_gbs": best_copy,
            "published": {"fp32_tflops": PEAK_FP32_TFLOPS, "hbm_gbs": PEAK_HBM_GBS},
            "method": f"FMA loop {n_blocks} x 256 lanes x 16 chains x {iters}; copy 1 GiB "
                      f"read + 1 GiB written; best of {reps}"}


def plain_vs_batched(dev, spec, params, n_bl=3, n_ap=4096, reps=5):
    """The one-window-per-launch path and the batched path on the same
    subset of the resident scan (baselines 0..n_bl-1, APs 0..n_ap-1)."""
    import torch

    import paper_2108_05602_amd as F
    sub = dev[:n_bl, :n_ap].contiguous()
    desc = dict(spec.desc(), n_baselines=n_bl, n_ap=n_ap)
    st = torch.cuda.current_stream()
    kw = dict(pad_freq=params["pad_freq"], pad_time=params["pad_time"],
              snr_threshold=params["snr_threshold"], max_candidates=1 << 20)
    out = {}
    for name, flags, n in (("plain", F.FRINGE_PLAIN, 1), ("batched", 0, reps)):
        with F.Plan([desc], params["window_aps"], flags=flags, **kw) as plan:
            plan.search([sub.data_ptr()], st.cuda_stream)
            plan.candidates()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n):
                plan.search([sub.data_ptr()], st.cuda_stream)
                plan.candidates()
            dt = (time.perf_counter() - t0) / n
            out[name] = plan.info()["n_windows"] / dt
            out["windows"] = plan.info()["n_windows"]
    out["speedup"] = out["batched"] / out["plain"]
    out["subset"] = f"baselines 0-{n_bl - 1} x APs 0-{n_ap - 1} of the same scan"
    return out


def delay_only_leg(dev, spec, params, steps=5):
    """The paper's own delay-only search (FRINGE_DELAY_ONLY: rate bin 0, the
    APs of each window summed, the peak over the delay axis) on the same
    resident scan and windows: windows/s and its kernel's time."""
    import torch

    import paper_2108_05602_amd as F
    st = torch.cuda.current_stream()
    with F.Plan([spec.desc()], params["window_aps"], pad_freq=params["pad_freq"],
                pad_time=params["pad_time"], snr_threshold=params["snr_threshold"],
                max_candidates=1 << 20, flags=F.FRINGE_DELAY_ONLY | F.FRINGE_PROFILE) as plan:
        n_win = plan.info()["n_windows"]
        for _ in range(2):
            plan.search([dev.data_ptr()], st.cuda_stream)
            plan.candidates()
        torch.cuda.synchronize()
        kern = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.search([dev.data_ptr()], st.cuda_stream)
            c = plan.candidates()
            kern += plan.profile()["rate_ms"]
        dt = (time.perf_counter() - t0) / steps
    m_f = params["pad_freq"] * spec.n_freq
    # algorithmic work: the delay FFT of every AP; per window and bin one
    # complex add (a window is the sum of its two halves; none for W = 1)
    # and the power, max and power sum
    flops = spec.n_baselines * spec.n_ap * 5.0 * m_f * math.log2(m_f)
    for w, s_, n in window_levels(spec.n_ap, params["window_aps"]):
        flops += spec.n_baselines * n * m_f * ((2.0 if w > 1 else 0.0) + 5.0)
    k_ms = kern / steps
    tf = flops / (k_ms * 1e-3) / 1e12
    return {"windows_per_s": n_win / dt, "ms_per_step": dt * 1e3, "kernel_ms": k_ms,
            "kernel_tflops_algorithmic": tf,
            "kernel_hbm_gbs_algorithmic": spec.nbytes() / (k_ms * 1e-3) / 1e9,
            "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / PEAK_FP32_TFLOPS},
            "candidates": int(len(c))}


def calibrated_leg(dev, spec, params, steps=5):
    """The full search of the same resident scan with calibration gains
    (fringe_set_gains): per baseline and channel a phasor removing an
    instrumental delay of up to 20 ns per IF, a phase and an amplitude
    scale, 6 of the 256 channels flagged; windows/s and the kernel's time."""
    import torch

    import paper_2108_05602_amd as F
    d = spec.desc()
    rng = np.random.default_rng(7)
    f = np.arange(spec.n_freq)
    n_if = d["n_if"]
    tau = rng.uniform(-20e-9, 20e-9, (spec.n_baselines, n_if))
    phi = rng.uniform(0, 2 * np.pi, (spec.n_baselines, n_if))
    per_f_tau = np.repeat(tau, d["n_chan"], axis=1)
    per_f_phi = np.repeat(phi, d["n_chan"], axis=1)
    g = rng.uniform(0.8, 1.2, (spec.n_baselines, spec.n_freq)) * np.exp(
        -1j * (2 * np.pi * f[None, :] * d["chan_width_hz"] * per_f_tau + per_f_phi))
    g[:, 100:106] = 0.0
    gains = torch.from_numpy(g.astype(np.complex64)).cuda()
    st = torch.cuda.current_stream()
    with F.Plan([d], params["window_aps"], pad_freq=params["pad_freq"],
                pad_time=params["pad_time"], snr_threshold=params["snr_threshold"],
                max_candidates=1 << 20, flags=F.FRINGE_PROFILE) as plan:
        plan.set_gains(0, gains.data_ptr())
        n_win = plan.info()["n_windows"]
        for _ in range(2):
            plan.search([dev.data_ptr()], st.cuda_stream)
            plan.candidates()
        torch.cuda.synchronize()
        kern = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.search([dev.data_ptr()], st.cuda_stream)
            c = plan.candidates()
            kern += plan.profile()["rate_ms"]
        dt = (time.perf_counter() - t0) / steps
    return {"windows_per_s": n_win / dt, "ms_per_step": dt * 1e3, "kernel_ms": kern / steps,
            "candidates": int(len(c))}


def single_pulse_leg(cands, spec, reps=20):
    """The candidate consumers on the timed search's candidates (host code):
    matching into single pulses (paper criteria: 2 window lengths, 5
    baselines) and one Eq. (2) solve with leave-one-out per pulse."""
    import paper_2108_05602_amd as F
    import synth
    t0 = time.perf_counter()
    for _ in range(reps):
        rows, n_p = F.fringe_match(cands, 2, 5)
    match_ms = (time.perf_counter() - t0) / reps * 1e3
    spans = {}
    for r in rows:
        lo, hi = spans.get(int(r["pulse"]), (1 << 62, -1))
        spans[int(r["pulse"])] = (min(lo, int(r["t_lo"])), max(hi, int(r["t_hi"])))
    found = sum(1 for q in spec.pulses
                if any(lo < q.start + q.width and q.start < hi for lo, hi in spans.values()))
    # localization timing: each pulse's delays against partials of a random
    # Earth-fixed array (the synthetic delays are not geometric, so only the
    # solve's cost is measured here, not its answer)
    rng = np.random.default_rng(0)
    st = rng.normal(0, 3e6, (spec.n_stations, 3))
    pairs = synth.baseline_pairs(spec.n_stations)
    b_xyz = np.array([st[j] - st[i] for i, j in pairs])
    da, dd = F.fringe_delay_partials(b_xyz, 1.0, 0.5, 0.6)
    t0 = time.perf_counter()
    n_solve = 0
    for pid in spans:
        sel = rows[rows["pulse"] == pid]
        bl = sel["baseline"]
        F.fringe_localize(sel["delay_s"], da[bl], dd[bl])
        n_solve += 1
    loc_ms = (time.perf_counter() - t0) * 1e3
    return {"candidates": int(len(cands)), "single_pulses": int(n_p), "rows": int(len(rows)),
            "injected": len(spec.pulses), "injected_found": int(found),
            "match_ms": match_ms, "localize_ms_total": loc_ms, "solves": n_solve,
            "host": "one CPU thread"}


def dm_search_leg(dev, spec, params, n_dm=20, dm_max=500.0, steps=2, delay_only=False):
    """A DM search of the same resident scan: n_dm trials (DM 0..dm_max,
    channels from 1.6 GHz up) as n_dm scans of one plan over the one cube,
    each with its dedispersion shifts; windows/s over all trials.  With
    delay_only, the paper's own dedispersed search (rate bin 0)."""
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    d = spec.desc()
    freqs = channel_freqs_hz(1.6e9, d["n_if"], d["n_chan"], d["chan_width_hz"])
    dms = np.linspace(0.0, dm_max, n_dm)
    shifts = [torch.from_numpy(dm_shifts(dm, freqs, d["ap_seconds"])).cuda() for dm in dms]
    st = torch.cuda.current_stream()
    with F.Plan([d] * n_dm, params["window_aps"], pad_freq=params["pad_freq"],
                pad_time=params["pad_time"], snr_threshold=params["snr_threshold"],
                max_candidates=1 << 22,
                flags=F.FRINGE_PROFILE | (F.FRINGE_DELAY_ONLY if delay_only else 0)) as plan:
        for s_, sh in enumerate(shifts):
            plan.set_shifts(s_, sh.data_ptr())
        n_win = plan.info()["n_windows"]
        ptrs = [dev.data_ptr()] * n_dm
        plan.search(ptrs, st.cuda_stream)
        plan.candidates()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kern = 0.0
        for _ in range(steps):
            plan.search(ptrs, st.cuda_stream)
            c = plan.candidates(capacity=1 << 22)
            kern += plan.profile()["rate_ms"]
        dt = (time.perf_counter() - t0) / steps
        launches = plan.profile()["rate_launches"]
    return {"dm_trials": n_dm, "dm_max": dm_max, "max_shift_aps": int(shifts[-1].max()),
            "windows": n_win, "windows_per_s": n_win / dt, "ms_per_step": dt * 1e3,
            "ms_per_dm_trial": dt * 1e3 / n_dm, "fused_kernel_ms": kern / steps,
            "fused_launches": launches, "candidates": int(len(c))}


def dm_prepass_leg(dev, spec, params, n_dm=20, dm_max=500.0, group=10, steps=2):
    """The paper's dedispersed delay-only search by the dedispersion pass
    (fringe_dedisperse): per group of trials, each trial's cube dedispersed
    into a buffer of its own, then one search of the group's buffers
    without shifts; windows/s over all trials, the pass timed alone too."""
    import torch

    import paper_2108_05602_amd as F
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    d = spec.desc()
    freqs = channel_freqs_hz(1.6e9, d["n_if"], d["n_chan"], d["chan_width_hz"])
    dms = np.linspace(0.0, dm_max, n_dm)
    shifts = [torch.from_numpy(dm_shifts(dm, freqs, d["ap_seconds"])).cuda() for dm in dms]
    bufs = [torch.empty_like(dev) for _ in range(group)]
    st = torch.cuda.current_stream()
    with F.Plan([d] * group, params["window_aps"], pad_freq=params["pad_freq"],
                pad_time=params["pad_time"], snr_threshold=params["snr_threshold"],
                max_candidates=1 << 22, flags=F.FRINGE_DELAY_ONLY | F.FRINGE_PROFILE) as plan:
        ptrs = [b_.data_ptr() for b_ in bufs]

        def step():
            n_c, kern = 0, 0.0
            for g0 in range(0, n_dm, group):
                for k in range(group):
                    F.fringe_dedisperse(dev.data_ptr(), ptrs[k], spec.n_baselines, spec.n_ap,
                                        spec.n_freq, shifts[g0 + k].data_ptr(), st.cuda_stream)
                plan.search(ptrs, st.cuda_stream)
                n_c += len(plan.candidates(capacity=1 << 22))
                kern += plan.profile()["rate_ms"]
            return n_c, kern

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            n_c, kern = step()
        dt = (time.perf_counter() - t0) / steps
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for k in range(group):
            F.fringe_dedisperse(dev.data_ptr(), ptrs[k], spec.n_baselines, spec.n_ap,
                                spec.n_freq, shifts[k].data_ptr(), st.cuda_stream)
        e1.record(st)
        e1.synchronize()
        pass_ms = e0.elapsed_time(e1) / group
        n_win = plan.info()["n_windows"] * (n_dm // group)
    del bufs
    return {"dm_trials": n_dm, "dm_max": dm_max, "group": group, "windows": n_win,
            "windows_per_s": n_win / dt, "ms_per_step": dt * 1e3,
            "ms_per_dm_trial": dt * 1e3 / n_dm, "pass_ms_per_trial": pass_ms,
            "pass_hbm_gbs": 2 * spec.nbytes() / (pass_ms * 1e-3) / 1e9,
            "fused_kernel_ms_per_trial": kern / n_dm, "candidates": int(n_c),
            "buffers_gb": group * spec.nbytes() / 1e9}


def graph_vs_eager(dev, spec, params, n_bl=15, n_ap=976, rounds=6, reps=50):
    """Per-search latency (search + candidates on the host) of a small batch
    plan launched eagerly and replayed from its HIP graph (FRINGE_GRAPH), on
    baselines 0..n_bl-1 x APs 0..n_ap-1 of the resident scan (a 1 s chunk of
    a 6-station array).  Both plans stay alive and are timed in alternating
    rounds; the medians of the rounds are reported."""
    import torch

    import paper_2108_05602_amd as F
    sub = dev[:n_bl, :n_ap].contiguous()
    desc = dict(spec.desc(), n_baselines=n_bl, n_ap=n_ap)
    st = torch.cuda.current_stream()
    kw = dict(pad_freq=params["pad_freq"], pad_time=params["pad_time"],
              snr_threshold=params["snr_threshold"], max_candidates=1 << 16)
    plans = {"eager": F.Plan([desc], params["window_aps"], **kw),
             "graph": F.Plan([desc], params["window_aps"], flags=F.FRINGE_GRAPH, **kw)}
    times = {k: [] for k in plans}
    try:
        for plan in plans.values():
            for _ in range(3):
                plan.search([sub.data_ptr()], st.cuda_stream)
                plan.candidates()
        for _ in range(rounds):
            for name, plan in plans.items():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    plan.search([sub.data_ptr()], st.cuda_stream)
                    plan.candidates()
                times[name].append((time.perf_counter() - t0) / reps * 1e6)
    finally:
        for plan in plans.values():
            plan.close()
    out = {"subset": f"baselines 0-{n_bl - 1} x APs 0-{n_ap - 1} of the same scan",
           "rounds": rounds, "reps_per_round": reps}
    for name, ts in times.items():
        out[name + "_us"] = float(np.median(ts))
    return out


class _Cycle:
    """payloads[seq] for any seq: a subarray's distinct chunks, repeated."""

    def __init__(self, chunks):
        self.chunks = chunks

    def __getitem__(self, i):
        return self.chunks[i % len(self.chunks)]


def serving_latency(n_sub=6, n_distinct=8, chunk_ap=976, chunks_per_point=600,
                    loads=(0.5, 1.0, 1.5, 2.0), time_chunks=(0, 128, 256, 336, 496), dm=100.0):
    """Streamed subarrays through the continuous-batching servers.

    Six subarrays of 3-12 stations (8 IF x 32 chan, 1.024 ms APs), chunks of
    976 APs (1 s) staged in HBM (each subarray's first n_distinct chunks,
    replayed in order).  Per server: the plans' time chunk is chosen by the
    saturated rate (every chunk queued at t = 0) of each candidate; R* = the
    rate served, in a run three times as long, while every subarray still
    has chunks waiting (up to the first subarray's last result: after it
    the GPU serves fewer subarrays than it was offered); then Poisson
    arrivals per subarray at x * R* / n_sub for each load x, and the p50 /
    p99 of arrival -> candidates-on-host latency.  `sustained_*` is the
    largest rate served over those runs, `served_vs_batch` its windows/s
    over those of one batch search of the same staged chunks.  The servers:
    the library's native one (primary: admission, launches and collection
    in its worker thread), the Python per-subarray one, and the
    one-launch-per-step one; further points: the native server with the
    subarrays dedispersed at DM `dm` (channels from 1.6 GHz), and the
    Python server fed from pinned host memory (H2D copy inside the
    latency)."""
    import torch

    import paper_2108_05602_amd as F
    import synth
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    from paper_2108_05602_amd.serve import (FringeBatchServer, FringeNativeServer, FringeServer,
                                            poisson_schedule, run_schedule)
    specs = synth.c4_subarrays(n_sub, n_chunks=n_distinct, chunk_ap=chunk_ap)
    dev, host, whole = [], [], []
    for s in specs:
        v = s.full(threads=min(16, os.cpu_count() or 1))
        t = torch.from_numpy(v)
        whole.append(t[:, :n_distinct * chunk_ap].contiguous().to("cuda:0"))
        dev.append([whole[-1][:, k * chunk_ap:(k + 1) * chunk_ap].contiguous()
                    for k in range(n_distinct)])
        host.append([t[:, k * chunk_ap:(k + 1) * chunk_ap].contiguous().pin_memory()
                     for k in range(min(2, n_distinct))])
        del v, t
    torch.cuda.synchronize()
    subs = [dict(s.desc(), n_ap=chunk_ap) for s in specs]
    per_sub = max(1, chunks_per_point // n_sub)
    out = {"subarrays": [s["n_baselines"] for s in subs], "chunk_ap": chunk_ap,
           "chunks_per_point": per_sub * n_sub,
           "staging": f"first {n_distinct} chunks of each subarray's stream resident in HBM, replayed"}

    def run(payloads, sched, server, steady=False, **kw):
        srv = server(subs, WS_C4, snr_threshold=4.5, **kw)
        try:
            run_schedule(srv, [(0.0, s, k) for s in range(n_sub) for k in range(2)], payloads)
            st = run_schedule(srv, sched, payloads)
        finally:
            srv.close()
        torch.cuda.synchronize()
        res = st.summary()
        if steady:
            # served while every subarray is busy: up to the first
            # subarray's last result (arrivals all at t = 0)
            t_end = min(max(r.done for r in st.results if r.sub == s) for s in range(n_sub))
            done = [r for r in st.results if r.done <= t_end]
            res["steady_s"] = t_end
            res["steady_chunks_per_s"] = len(done) / t_end
            res["steady_windows_per_s"] = sum(r.n_windows for r in done) / t_end
        return res

    def burst(n):
        return [(0.0, s, k) for s in range(n_sub) for k in range(n)]

    pd = [_Cycle(c) for c in dev]
    # the same staged chunks as one batch search (whole streams, one plan)
    st = torch.cuda.current_stream()
    bdesc = [dict(s.desc(), n_ap=n_distinct * chunk_ap) for s in specs]
    with F.Plan(bdesc, WS_C4, snr_threshold=4.5) as bp:
        ptrs = [w.data_ptr() for w in whole]
        for _ in range(2):
            bp.search(ptrs, st.cuda_stream)
            bp.candidates()
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bp.search(ptrs, st.cuda_stream)
            bp.candidates()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        b_wps = bp.info()["n_windows"] / float(np.median(ts))
    out["batch_windows_per_s"] = b_wps

    def measure(server, label, **kw):
        sweep = {}
        for c in time_chunks:
            sweep[c] = run(pd, burst(per_sub), server, time_chunk=c, **kw)["chunks_per_s"]
            log(f"serving ({label}) time chunk {c or 'auto'}: {sweep[c]:.0f} chunks/s saturated")
        tc = max(sweep, key=sweep.get)
        sat = run(pd, burst(3 * per_sub), server, steady=True, time_chunk=tc, **kw)
        r_star = sat["steady_chunks_per_s"]
        m = {"time_chunk": {"chosen": tc,
                            "saturated_chunks_per_s": {str(k): v for k, v in sweep.items()}},
             "saturated": sat, "r_star_chunks_per_s": r_star, "points": []}
        for x in loads:
            p = run(pd, poisson_schedule(n_sub, per_sub, x * r_star / n_sub, seed=int(x * 100)),
                    server, time_chunk=tc, **kw)
            p["load"] = x
            m["points"].append(p)
            log(f"serving ({label}) load {x}: p50 {p['p50_ms']:.3f} ms, p99 {p['p99_ms']:.3f} ms, "
                f"{p['chunks_per_s']:.0f} chunks/s")
        rates = [(sat["steady_chunks_per_s"], sat["steady_windows_per_s"])] + \
            [(p["chunks_per_s"], p["windows_per_s"]) for p in m["points"]]
        best = max(rates, key=lambda r: r[1])
        m["sustained_chunks_per_s"], m["served_windows_per_s"] = best
        m["served_vs_batch"] = best[1] / b_wps
        log(f"serving ({label}): R* {r_star:.0f} chunks/s, sustained {best[0]:.0f} chunks/s, "
            f"{best[1] / 1e6:.1f} M windows/s = {m['served_vs_batch']:.2f} of batch "
            f"({b_wps / 1e6:.1f} M windows/s)")
        return m

    nat = measure(FringeNativeServer, "native")
    out.update(nat)
    out["server"] = "FringeNativeServer (library worker thread)"
    out["python"] = measure(FringeServer, "python")
    tc = nat["time_chunk"]["chosen"]
    # dedispersed serving: every subarray at one DM, native server
    shifts = []
    for sd in subs:
        f = channel_freqs_hz(1.6e9, sd["n_if"], sd["n_chan"], sd["chan_width_hz"])
        shifts.append(torch.from_numpy(dm_shifts(dm, f, sd["ap_seconds"])).to("cuda:0"))
    dsat = run(pd, burst(3 * per_sub), FringeNativeServer, steady=True, time_chunk=tc, shifts=shifts)
    dpt = run(pd, poisson_schedule(n_sub, per_sub, dsat["steady_chunks_per_s"] / n_sub, seed=11),
              FringeNativeServer, time_chunk=tc, shifts=shifts)
    dpt["load"] = 1.0
    out["dedispersed"] = {"dm": dm, "max_shift_ap": int(max(int(x.max()) for x in shifts)),
                          "r_star_chunks_per_s": dsat["steady_chunks_per_s"], "saturated": dsat,
                          "point": dpt}
    log(f"serving (native) at DM {dm}: R* {dsat['steady_chunks_per_s']:.0f} chunks/s, p50 "
        f"{dpt['p50_ms']:.3f} ms, p99 {dpt['p99_ms']:.3f} ms at that load")
    # pinned host chunks (H2D copy inside the latency), Python server
    tcp = out["python"]["time_chunk"]["chosen"]
    ph = [_Cycle(c) for c in host]
    hs = run(ph, burst(per_sub), FringeServer, time_chunk=tcp)
    hp = run(ph, poisson_schedule(n_sub, per_sub, 0.5 * hs["chunks_per_s"] / n_sub, seed=7),
             FringeServer, time_chunk=tcp)
    hp["load"] = 0.5
    out["pinned_host"] = {"r_star_chunks_per_s": hs["chunks_per_s"], "point": hp}
    # one launch per step over all waiting subarrays
    bsat = run(pd, burst(3 * per_sub), FringeBatchServer, steady=True, time_chunk=tcp)
    out["batched"] = {"r_star_chunks_per_s": bsat["steady_chunks_per_s"], "saturated": bsat,
                      "points": []}
    for x in loads:
        p = run(pd, poisson_schedule(n_sub, per_sub, x * nat["r_star_chunks_per_s"] / n_sub,
                                     seed=int(x * 100)), FringeBatchServer, time_chunk=tcp)
        p["load"] = x
        out["batched"]["points"].append(p)
        log(f"serving (batched) load {x} of the native R*: p50 {p['p50_ms']:.3f} ms, "
            f"p99 {p['p99_ms']:.3f} ms, {p['chunks_per_s']:.0f} chunks/s")
    return out


WS_C4 = [1, 2, 4, 8, 16, 32]

C3_WORKLOAD = ("Batched uneven: 200 scans of 10-120 s (1.024 ms APs), 3-12 stations (3-66 baselines), "
               "8 or 16 IF x {16,32,64} chan complex64 (16 MHz IFs), pulses and narrowband RFI, "
               "windows 1-64 AP at 50% overlap, 4x delay / 2x rate padding, SNR > 4.5; generated on "
               "the device in HBM-budgeted waves, one plan per wave")


def c3_headline(steps, warmup, wave_gb, n_scans=200, cpu_sample=None, autotune=True,
                compare_default=True, tune_load=None, tune_save=None):
    """The batched uneven workload: per wave, generate its scans on the
    device, build one plan, search it `warmup` times untimed and `steps`
    times timed (each search with its candidate copy, bracketed by device
    synchronisations).  Step k's time is the sum over the waves of their
    k-th timed search.  cpu_sample, if a list, receives host copies of a
    few baselines' first APs from one scan of each band width (the CPU
    reference's sample of this workload).  tune_load: a tune table file
    read instead of tuning (no timing launches in the run); tune_save: where
    to write the table afterwards."""
    import torch

    import paper_2108_05602_amd as F
    import synth
    from synth import device as sd
    specs = synth.c3(n_scans=n_scans)
    p = synth.C3_PARAMS
    groups = sd.waves(specs, int(wave_gb * 1e9))
    st = torch.cuda.current_stream()
    flags = F.FRINGE_PROFILE | (F.FRINGE_AUTOTUNE if autotune else 0)
    if autotune:
        F.fringe_tune_clear()
        if tune_load:
            F.fringe_tune_load(tune_load)
    plan_s = 0.0
    entries = {}
    cmp = None
    step_s = [0.0] * steps
    fused_ms = fin_ms = comp_ms = delay_ms = 0.0
    fused_n = delay_n = 0
    n_windows = n_cands = cube = 0
    fl = [0.0, 0.0, 0.0]
    part_bytes = e_bytes = 0
    # per kernel: the fused search kernel (all its instantiations) and the
    # delay transform of bands in spectra mode: algorithmic flops and bytes
    k_fl = {"fused": 0.0, "delay": 0.0}
    k_by = {"fused": 0.0, "delay": 0.0}
    sampled_f = set()
    waves_out = []
    log(f"C3: {len(specs)} scans, {sum(s.nbytes() for s in specs) / 1e12:.3f} TB in "
        f"{len(groups)} waves of <= {wave_gb} GB")
    for wi, idx in enumerate(groups):
        t0 = time.perf_counter()
        tens = [sd.generate(specs[i]) for i in idx]
        torch.cuda.synchronize()
        gen_s = time.perf_counter() - t0
        descs = [specs[i].desc() for i in idx]
        t0 = time.perf_counter()
        with F.Plan(descs, p["window_aps"], pad_freq=p["pad_freq"], pad_time=p["pad_time"],
                    snr_threshold=p["snr_threshold"], max_candidates=1 << 22,
                    flags=flags) as plan:
            plan_s += time.perf_counter() - t0
            if autotune:
                for e in plan.tuning():
                    entries[e["n_freq"]] = e
            ptrs = [t.data_ptr() for t in tens]
            for _ in range(warmup):
                plan.search(ptrs, st.cuda_stream)
                plan.candidates()
            wt = []
            for k in range(steps):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                plan.search(ptrs, st.cuda_stream)
                c = plan.candidates()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                step_s[k] += dt
                wt.append(dt)
                pr = plan.profile()
                fused_ms += pr["rate_ms"]
                fused_n += pr["rate_launches"]
                delay_ms += pr["delay_ms"]
                delay_n += pr["delay_launches"]
                fin_ms += pr["finalize_ms"]
                comp_ms += pr["compact_ms"]
            nw = plan.info()["n_windows"]
        if autotune and compare_default and wi == 0:
            # the same wave with the default configurations, timed alike
            with F.Plan(descs, p["window_aps"], pad_freq=p["pad_freq"], pad_time=p["pad_time"],
                        snr_threshold=p["snr_threshold"], max_candidates=1 << 22,
                        flags=F.FRINGE_PROFILE) as dplan:
                dplan.search(ptrs, st.cuda_stream)
                dplan.candidates()
                dt_def = []
                for _ in range(max(2, min(steps, 5))):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    dplan.search(ptrs, st.cuda_stream)
                    dplan.candidates()
                    torch.cuda.synchronize()
                    dt_def.append(time.perf_counter() - t1)
            cmp = {"wave": 0, "scans": len(idx), "default_ms": float(np.median(dt_def)) * 1e3,
                   "tuned_ms": float(np.median(wt)) * 1e3}
            cmp["gain"] = cmp["default_ms"] / cmp["tuned_ms"]
            log(f"C3 wave 0, default configurations: {cmp['default_ms']:.1f} ms vs tuned "
                f"{cmp['tuned_ms']:.1f} ms")
        n_windows += nw
        n_cands += len(c)
        wb = 0
        for i in idx:
            sp = specs[i]
            d_, r_, k_ = algorithmic_flops(sp.n_baselines, sp.n_ap, sp.n_freq, p["window_aps"],
                                           p["pad_freq"], p["pad_time"])
            fl[0] += d_
            fl[1] += r_
            fl[2] += k_
            wb += sp.nbytes()
            n_cls = p["pad_freq"] * sp.n_freq // 64
            nw_s = sum(n for _, _, n in window_levels(sp.n_ap, p["window_aps"])) * sp.n_baselines
            part_bytes += nw_s * n_cls * 8
            e_bytes += sp.n_baselines * sp.n_ap * 4
            # the band's search mode: the tuned one, else the default (spectra
            # for bands of more than 512 channels)
            spectra = (entries[sp.n_freq]["spectra"] if sp.n_freq in entries
                       else int(sp.n_freq > 512))
            x_bytes = sp.n_baselines * sp.n_ap * p["pad_freq"] * sp.n_freq * 8
            if spectra:
                k_fl["fused"] += r_ + k_
                k_fl["delay"] += d_
                k_by["fused"] += x_bytes + nw_s * n_cls * 8
                k_by["delay"] += sp.nbytes() + x_bytes + sp.n_baselines * sp.n_ap * 4
            else:
                k_fl["fused"] += d_ + r_ + k_
                k_by["fused"] += sp.nbytes() + nw_s * n_cls * 8 + sp.n_baselines * sp.n_ap * 4
        cube += wb
        if cpu_sample is not None:
            for j, i in enumerate(idx):
                sp = specs[i]
                if sp.n_freq in sampled_f:
                    continue
                sampled_f.add(sp.n_freq)
                t_n = min(4096, sp.n_ap)
                for b in range(min(3, sp.n_baselines)):
                    cpu_sample.append((i, b, sp, tens[j][b, :t_n].reshape(t_n, -1).cpu().numpy()))
        waves_out.append({"scans": len(idx), "gb": wb / 1e9, "windows": nw, "candidates": int(len(c)),
                          "gen_s": gen_s, "search_ms_median": float(np.median(wt)) * 1e3})
        log(f"C3 wave {wi}: {len(idx)} scans, {wb / 1e9:.1f} GB, {nw} windows, generated in "
            f"{gen_s:.1f} s, search {np.median(wt) * 1e3:.1f} ms, {len(c)} candidates")
        del tens
        torch.cuda.empty_cache()
    if autotune and tune_save:
        F.fringe_tune_save(tune_save)
    ms = float(np.mean(step_s)) * 1e3
    flops_step = fl[0] + fl[1] + fl[2]
    # the search kernels of a step: the fused kernels (delay transform, rate
    # transform and peak in one) and, for bands in spectra mode, the delay
    # transform kernel and the fused kernel reading its spectra; their
    # algorithmic flops over their summed launch time
    launches_per_step = (fused_n + delay_n) / steps
    avg_launch_s = (fused_ms + delay_ms) / max(1, fused_n + delay_n) / 1e3
    flops_per_launch = flops_step / launches_per_step
    achieved = flops_per_launch / avg_launch_s / 1e12
    # the dominant kernel: the fused search kernel, every instantiation
    # (fused-mode bands: delay + rate transforms + peaks; spectra-mode bands:
    # rate transforms + peaks from the spectra)
    fk_n = fused_n / steps
    fk_s = fused_ms / max(1, fused_n) / 1e3
    fk_achieved = k_fl["fused"] / fk_n / fk_s / 1e12
    dk_n = delay_n / steps
    dk_s = delay_ms / max(1, delay_n) / 1e3 if delay_n else None
    mt = MEASURED_TRAFFIC_C3
    tuned = {k: (v["spectra"], v["chunk"]) for k, v in entries.items()}
    valid = (n_scans == 200 and autotune and tuned == mt["tuning"] and
             fk_n == mt["fused_launches_per_step"] and dk_n == mt["delay_launches_per_step"] and
             kernel_hash(C3_SOURCES) == mt["kernel_sha256"])
    traffic = traffic_all = traffic_delay = None
    if valid:
        traffic = (mt["fused_fetch_bytes"] + mt["fused_write_bytes"]) / fk_n
        traffic_delay = (mt["delay_fetch_bytes"] + mt["delay_write_bytes"]) / dk_n
        traffic_all = (mt["fused_fetch_bytes"] + mt["fused_write_bytes"] + mt["delay_fetch_bytes"] +
                       mt["delay_write_bytes"]) / launches_per_step
    return {
        "value": n_windows / (ms / 1e3), "ms_per_step": ms, "windows": n_windows, "cube_bytes": cube,
        "candidates": n_cands, "waves": waves_out, "scans": len(specs),
        "roofline": {
            "bound": "alu",
            "kernel": "fused_search_kernel, every instantiation: delay FFT + rate FFT + |G|^2 peak "
                      "for bands in fused mode (one launch per wave and fold class), rate FFT + "
                      "|G|^2 peak from the delay spectra for bands in spectra mode (one launch "
                      "per baseline slab)",
            "achieved": fk_achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": fk_achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "algorithmic_flops_per_launch": k_fl["fused"] / fk_n,
            "algorithmic_bytes_per_launch": k_by["fused"] / fk_n,
            "avg_launch_ms": fk_s * 1e3,
            "launches_per_step": fk_n,
        },
        "roofline_delay_fft": None if not delay_n else {
            "bound": "hbm",
            "kernel": "delay_fft_kernel (bands in spectra mode: visibilities in, delay spectra out)",
            "achieved": k_by["delay"] / dk_n / dk_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": k_by["delay"] / dk_n / dk_s / 1e9 / PEAK_HBM_GBS,
            "traffic": traffic_delay,
            "algorithmic_bytes_per_launch": k_by["delay"] / dk_n,
            "algorithmic_flops_per_launch": k_fl["delay"] / dk_n,
            "avg_launch_ms": dk_s * 1e3, "launches_per_step": dk_n,
        },
        "search_kernels": {
            "kernels": "fused_search_kernel and delay_fft_kernel together",
            "achieved_tflops": achieved, "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic_per_launch": traffic_all,
            "algorithmic_flops_per_launch": flops_per_launch,
            "algorithmic_bytes_per_launch": (cube + part_bytes + e_bytes) / launches_per_step,
            "avg_launch_ms": avg_launch_s * 1e3, "launches_per_step": launches_per_step,
        },
        "kernel_ms_per_step": {"fused_ms": fused_ms / steps, "delay_fft_ms": delay_ms / steps,
                               "finalize_ms": fin_ms / steps, "compact_ms": comp_ms / steps},
        "tflops_algorithmic_step": flops_step / (ms / 1e3) / 1e12,
        "hbm_gbs_algorithmic": cube / (ms / 1e3) / 1e9,
        "hbm_gbs_measured": (None if traffic_all is None else
                             traffic_all * launches_per_step / (ms / 1e3) / 1e9),
        "autotune": {"enabled": autotune, "plan_s_total": plan_s,
                     "table": os.path.relpath(tune_load, ROOT) if tune_load else "tuned in this run",
                     "entries": [entries[k] for k in sorted(entries)],
                     "tuned_vs_default": cmp},
    }


def cpu_baseline_c3(sample, params):
    """The CPU reference, as it stands, on the headline workload's sample:
    baselines 0-2 x the first 4,096 APs of the first scan of each band
    width (copied from the device-generated cubes), every window length;
    with numpy's BLAS pool (the reported value) and, on the narrowest of
    them, one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import fringe_oracle as fo

    def run(items):
        n = 0
        t0 = time.perf_counter()
        for i, b, sp, x in items:
            n += len(fo.search_baseline(x, params["window_aps"], params["pad_freq"],
                                        params["pad_time"], sp.ap_seconds, sp.chan_width_hz,
                                        scan=i, baseline=b))
        return n, time.perf_counter() - t0

    n, dt = run(sample)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        n1, dt1 = run(sample[:1])
    desc = "; ".join(f"scan {i} (F = {sp.n_freq}) baseline {b} x APs 0-{x.shape[0] - 1}"
                     for i, b, sp, x in sample)
    return {"value": n / dt, "unit": "windows/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{desc}: {n} windows in {dt:.1f} s",
            "one_thread": {"value": n1 / dt1, "sample": f"the first of these: {n1} windows in "
                                                        f"{dt1:.1f} s"}}


def large_dense_leg(steps=2, warmup=1):
    """The large dense scan (66 BL x 117,200 AP x 1,024 chan, 63.4 GB,
    windows 1-128 APs), generated on the device: windows/s of full
    searches and each kernel's time and algorithmic rate."""
    import torch

    import paper_2108_05602_amd as F
    import synth
    from synth import device as sd
    spec = synth.c5()
    p = synth.C5_PARAMS
    t0 = time.perf_counter()
    dev = sd.generate(spec)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    st = torch.cuda.current_stream()
    with F.Plan([spec.desc()], p["window_aps"], pad_freq=p["pad_freq"], pad_time=p["pad_time"],
                snr_threshold=p["snr_threshold"], max_candidates=1 << 22,
                flags=F.FRINGE_PROFILE) as plan:
        for _ in range(warmup):
            plan.search([dev.data_ptr()], st.cuda_stream)
            plan.candidates()
        ts, prof = [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan.search([dev.data_ptr()], st.cuda_stream)
            c = plan.candidates()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
            prof.append(plan.profile())
        n_win = plan.info()["n_windows"]
        slab = plan.info()["slab_baselines"]
    del dev
    torch.cuda.empty_cache()
    dt = float(np.mean(ts))
    pr = {k: float(np.mean([q[k] for q in prof])) for k in prof[0]}
    m_f = p["pad_freq"] * spec.n_freq
    nb, T = spec.n_baselines, spec.n_ap
    short = [w for w in p["window_aps"] if w <= 64]
    long_ = [w for w in p["window_aps"] if w > 64]
    d_fl, r_s, k_s = algorithmic_flops(nb, T, spec.n_freq, short, p["pad_freq"], p["pad_time"])
    _, r_l, k_l = algorithmic_flops(nb, T, spec.n_freq, long_, p["pad_freq"], p["pad_time"])
    total = d_fl + r_s + k_s + r_l + k_l
    return {"workload": "large dense scan: 66 BL x 117200 AP (0.512 ms) x 16 IF x 64 chan complex64, "
                        "windows 1-128 AP, 63.4 GB, generated on the device",
            "windows": n_win, "windows_per_s": n_win / dt, "ms_per_search": dt * 1e3,
            "generate_s": gen_s, "slab_baselines": slab, "candidates": int(len(c)),
            "kernel_ms": {"delay_fft": pr["delay_ms"], "fused_and_rate": pr["rate_ms"],
                          "finalize": pr["finalize_ms"], "compact": pr["compact_ms"]},
            "launches": {"delay_fft": pr["delay_launches"], "fused_and_rate": pr["rate_launches"]},
            "tflops_algorithmic": total / dt / 1e12,
            "frac_fp32_peak": total / dt / 1e12 / PEAK_FP32_TFLOPS,
            "delay_fft_hbm_gbs": (nb * T * (spec.n_freq + m_f) * 8) / (pr["delay_ms"] * 1e-3) / 1e9
            if pr["delay_ms"] > 0 else None}


def calibration_copy(mib):
    """One device-to-device copy of `mib` MiB: a plain copy kernel of known
    size, for scaling hardware byte counters."""
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy: {n} bytes read, {n} bytes written")
    del src, dst
    torch.cuda.empty_cache()


def evn_scan_legs(args, out):
    """The EVN-like single scan: its own search (5 steps), then the legs
    that compare paths on it."""
    import torch

    import paper_2108_05602_amd as F
    import synth
    params = dict(synth.C2_PARAMS)
    spec = synth.c2(n_stations=args.stations, n_ap=args.n_ap)
    full = args.stations == 10 and args.n_ap == 58600
    log(f"EVN scan: generating {spec.n_baselines} BL x {spec.n_ap} AP x {spec.n_freq} ch "
        f"({spec.nbytes() / 1e9:.2f} GB)")
    v = spec.full(threads=min(16, os.cpu_count() or 1))
    dev = torch.from_numpy(v).to("cuda:0")
    del v
    torch.cuda.synchronize()
    if args.calibrate_copy and args.only == "c2":
        calibration_copy(args.calibrate_copy)
    steps = args.evn_steps
    plan = F.Plan([spec.desc()], params["window_aps"], pad_freq=params["pad_freq"],
                  pad_time=params["pad_time"], snr_threshold=params["snr_threshold"],
                  max_candidates=1 << 20, flags=F.FRINGE_PROFILE)
    n_win = plan.info()["n_windows"]
    stream = torch.cuda.current_stream()
    for _ in range(2):
        plan.search([dev.data_ptr()], stream.cuda_stream)
        plan.candidates()
    torch.cuda.synchronize()
    kern = {"delay_ms": 0.0, "rate_ms": 0.0, "finalize_ms": 0.0, "compact_ms": 0.0}
    launches = 0
    t_wall = time.perf_counter()
    for _ in range(steps):
        plan.search([dev.data_ptr()], stream.cuda_stream)
        cands = plan.candidates()
        prof = plan.profile()
        for k in kern:
            kern[k] += prof[k]
        launches += prof["rate_launches"]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t_wall) / steps * 1e3
    plan.close()
    d_fl, r_fl, p_fl = algorithmic_flops(spec.n_baselines, spec.n_ap, spec.n_freq,
                                         params["window_aps"], params["pad_freq"], params["pad_time"])
    avg_launch_s = kern["rate_ms"] / max(1, launches) / 1e3
    flops_per_launch = (d_fl + r_fl + p_fl) * steps / max(1, launches)
    achieved = flops_per_launch / avg_launch_s / 1e12
    n_cls = params["pad_freq"] * spec.n_freq // 64
    traffic = None
    if full and kernel_hash() == MEASURED_TRAFFIC["kernel_sha256"]:
        traffic = MEASURED_TRAFFIC["fetch_bytes"] + MEASURED_TRAFFIC["write_bytes"]
    ev = {"workload": ("EVN-like single scan: 45 baselines x 58600 AP x 8 IF x 32 chan complex64, "
                       "windows 1-32 AP at 50% overlap, 4x delay / 2x rate padding, SNR > 4.5")
          if full else f"reduced EVN-like scan: {spec.n_baselines} BL x {spec.n_ap} AP (quick check)",
          "windows": n_win, "cube_bytes": spec.nbytes(), "windows_per_s": n_win / (ms / 1e3),
          "ms_per_step": ms, "steps": steps,
          "kernel_ms_per_step": {k: x / steps for k, x in kern.items()},
          "candidates": int(len(cands)),
          "roofline": {"bound": "alu", "kernel": "fused_search_kernel<2, 5, 4>",
                       "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                       "algorithmic_flops_per_launch": flops_per_launch,
                       "algorithmic_bytes_per_launch": spec.nbytes() + n_win * n_cls * 8 +
                       spec.n_baselines * spec.n_ap * 4,
                       "avg_launch_ms": avg_launch_s * 1e3}}
    out["evn_scan"] = ev
    log("EVN scan: " + json.dumps({k: ev[k] for k in ("windows_per_s", "ms_per_step")}))
    if not args.no_plain:
        log("timing the one-window-per-launch path against the batched path")
        ev["plain_vs_batched"] = plain_vs_batched(dev, spec, params)
        log("plain vs batched: " + json.dumps(ev["plain_vs_batched"]))
    log("single pulses from the candidates (host matching and localization)")
    ev["single_pulses"] = single_pulse_leg(cands, spec)
    log("calibrated search of the same scan")
    ev["calibrated"] = calibrated_leg(dev, spec, params)
    log("delay-only search of the same scan")
    ev["delay_only"] = delay_only_leg(dev, spec, params)
    log("delay-only: " + json.dumps(ev["delay_only"]))
    log("DM search: 20 dedispersed trials of the same scan in one plan")
    ev["dm_search"] = dm_search_leg(dev, spec, params)
    log("DM search, delay-only (the paper's dedispersed search)")
    ev["dm_search_delay_only"] = dm_search_leg(dev, spec, params, delay_only=True)
    log("DM search, delay-only, by the dedispersion pass")
    ev["dm_search_delay_only_pass"] = dm_prepass_leg(dev, spec, params)
    log("small batch plan: eager launches vs graph replay")
    ev["graph_vs_eager"] = graph_vs_eager(dev, spec, params)
    if not args.no_cpu_baseline:
        log("timing the CPU reference on the EVN scan's sample")
        ev["cpu_baseline"] = cpu_baseline(spec, params)
    del dev
    torch.cuda.empty_cache()
    return ev


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", choices=["c3", "c2", "c5"], default=None,
                    help="run only the headline (c3), only the EVN-scan legs (c2) or only "
                         "the large dense scan (c5)")
    ap.add_argument("--wave-gb", type=float, default=150.0,
                    help="visibilities per wave of the headline workload")
    ap.add_argument("--c3-scans", type=int, default=200, help="(fewer: quick check only)")
    ap.add_argument("--evn-steps", type=int, default=5)
    ap.add_argument("--stations", type=int, default=10, help="EVN scan (smaller: quick check only)")
    ap.add_argument("--n-ap", type=int, default=58600, help="EVN scan (smaller: quick check only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="headline plans with the default configurations (no tuning)")
    ap.add_argument("--tune-load", metavar="JSON", default=None,
                    help="headline: read this tune table instead of tuning (default: the "
                         "table shipped for MI355X, %s)" % os.path.relpath(SHIPPED_TUNE, ROOT))
    ap.add_argument("--retune", action="store_true",
                    help="headline: tune every class afresh instead of reading a table")
    ap.add_argument("--tune-save", metavar="JSON", default=None,
                    help="headline: write the tune table here afterwards")
    ap.add_argument("--no-compare-default", action="store_true",
                    help="headline: skip timing wave 0 with the default configurations")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the first search, copy a MIB-MiB device buffer once (a plain "
                         "copy kernel of known size for scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2108_05602_amd as F
    import synth
    F.load()
    torch.cuda.init()

    out = {"metric": "fringe-fit windows/s + HBM GB/s vs roofline; p50/p99 window latency",
           "unit": "windows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}
    sample = []
    if args.only == "c5":
        if args.calibrate_copy:
            calibration_copy(args.calibrate_copy)
        ld = large_dense_leg(steps=args.steps, warmup=args.warmup)
        out["value"] = ld["windows_per_s"]
        out["ms_per_step"] = ld["ms_per_search"]
        out["config"] = {"workload": ld["workload"], "windows": ld["windows"],
                         "parallelism": "single GPU"}
        out["large_dense"] = ld
        print(json.dumps(out), flush=True)
        return
    if args.calibrate_copy and args.only != "c2":
        calibration_copy(args.calibrate_copy)
    if args.only != "c2":
        h = c3_headline(args.steps, args.warmup, args.wave_gb, n_scans=args.c3_scans,
                        cpu_sample=None if args.no_cpu_baseline else sample,
                        autotune=not args.no_autotune,
                        compare_default=not args.no_compare_default,
                        tune_load=None if args.retune else (args.tune_load or SHIPPED_TUNE),
                        tune_save=args.tune_save)
        out["value"] = h["value"]
        out["ms_per_step"] = h["ms_per_step"]
        out["config"] = {"workload": C3_WORKLOAD if args.c3_scans == 200 else
                         f"reduced batched uneven set: first {args.c3_scans} scans (quick check)",
                         "scans": h["scans"], "windows": h["windows"], "cube_bytes": h["cube_bytes"],
                         "waves": len(h["waves"]), "parallelism": "single GPU"}
        out["roofline"] = h["roofline"]
        for k in ("roofline_delay_fft", "search_kernels", "kernel_ms_per_step",
                  "tflops_algorithmic_step", "hbm_gbs_algorithmic", "hbm_gbs_measured",
                  "candidates", "waves", "autotune"):
            out[k] = h[k]
        out["hbm_frac_algorithmic"] = h["hbm_gbs_algorithmic"] / PEAK_HBM_GBS
        log(f"C3 headline: {h['value'] / 1e6:.1f} M windows/s, {h['ms_per_step']:.1f} ms per step, "
            f"fused kernels {h['roofline']['achieved']:.1f} TFLOP/s")
    if args.only != "c3":
        ev = evn_scan_legs(args, out)
        if args.only == "c2":
            out["value"] = ev["windows_per_s"]
            out["ms_per_step"] = ev["ms_per_step"]
            out["steps"] = ev["steps"]
            out["config"] = {"workload": ev["workload"], "windows": ev["windows"],
                             "cube_bytes": ev["cube_bytes"], "parallelism": "single GPU"}
            out["roofline"] = ev["roofline"]
        if not args.no_large:
            log("large dense scan (generated on the device)")
            out["large_dense"] = large_dense_leg()
            log("large dense: " + json.dumps(out["large_dense"]))
        if not args.no_serving:
            log("serving: streamed subarrays, saturated rate and Poisson loads")
            out["serving"] = serving_latency()
            pts = out["serving"]["points"]
            out["p50_ms"] = next(p["p50_ms"] for p in pts if p["load"] == 1.0)
            out["p99_ms"] = next(p["p99_ms"] for p in pts if p["load"] == 1.0)
        log("roof probes: FP32 FMA loop and HBM copy")
        out["roofs_measured"] = roof_probes()
        out["roofline"]["frac_of_measured_peak"] = (out["roofline"]["achieved"] /
                                                    out["roofs_measured"]["fp32_fma_tflops"])
        log("roofs: " + json.dumps(out["roofs_measured"]))
    if sample:
        log("timing the CPU reference on the headline workload's sample")
        out["cpu_baseline"] = cpu_baseline_c3(sample, synth.C3_PARAMS)
        log("cpu baseline: " + json.dumps(out["cpu_baseline"]))
    elif args.only == "c2" and "cpu_baseline" in out.get("evn_scan", {}):
        out["cpu_baseline"] = out["evn_scan"]["cpu_baseline"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
