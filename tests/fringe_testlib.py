"""Helpers shared by the GPU parity tests: run the HIP path on a cube and
compare its per-window table and candidate list with the CPU reference.

Comparison rules (the tolerance is the FP32 bar of 1e-4 relative):
  * window keys (scan, baseline, window_ap, t_start) and the candidate order
    are exact;
  * the peak bin is exact, except in an ambiguous window, where the top two
    grid powers of the reference differ by less than 1e-4 relative: there
    the HIP bin must hold a reference power within 1e-4 of the maximum;
  * amp, SNR and energy agree to 1e-4 relative (absolute near zero);
  * a window may be in one candidate list and not the other only if its
    reference SNR is within 1e-4 relative of the threshold.
"""

from __future__ import annotations

import math

import numpy as np

import oracle.fringe_oracle as fo

RTOL = 1e-4


def to_device(vis: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(vis)).to("cuda")


def run_gpu(scans, vis_list, window_aps, pad_freq, pad_time, snr_threshold,
            max_candidates=1 << 16, flags=0, all_windows=True, gains=None):
    """Plan + search on cuda:0; returns (plan, table or None, candidates).
    gains: None, or per scan None / a (B, F) complex array."""
    import torch

    import paper_2108_05602_amd as F
    tensors = [to_device(v) for v in vis_list]
    plan = F.Plan(scans, window_aps, pad_freq=pad_freq, pad_time=pad_time,
                  snr_threshold=snr_threshold, max_candidates=max_candidates, flags=flags)
    g_dev = []
    if gains is not None:
        for s, g in enumerate(gains):
            if g is None:
                continue
            d = scans[s]
            g = np.ascontiguousarray(np.asarray(g, dtype=np.complex64))
            assert g.shape == (d["n_baselines"], d["n_if"] * d["n_chan"])
            g_dev.append(to_device(g))
            plan.set_gains(s, g_dev[-1].data_ptr())
    plan.search([t.data_ptr() for t in tensors], torch.cuda.current_stream().cuda_stream)
    cands = plan.candidates()
    table = None
    if all_windows:
        n = plan.info()["n_windows"]
        table = plan.windows(np.arange(n, dtype=np.int64)) if n else np.zeros(0, cands.dtype)
    torch.cuda.synchronize()
    del tensors
    del g_dev
    return plan, table, cands


def oracle_power_at(x_b, t0, w, pad_freq, pad_time, k_t, k_f):
    """Reference |G|^2 at one bin, by the direct double sum."""
    seg = np.asarray(x_b[t0:t0 + w], dtype=np.complex128)
    nf = seg.shape[1]
    m_t, m_f = pad_time * w, pad_freq * nf
    u = np.arange(w)[:, None]
    f = np.arange(nf)[None, :]
    g = np.sum(seg * np.exp(-2j * np.pi * (k_t * u / m_t + k_f * f / m_f)))
    return float(abs(g) ** 2)


def compare_windows(gpu, ref, x_by_baseline, pad_freq, pad_time, label=""):
    """Row-by-row comparison of HIP records with reference records (same
    windows, same order).  x_by_baseline(scan, b) gives (T, F) samples.
    Returns the number of ambiguous windows."""
    assert len(gpu) == len(ref), f"{label}: {len(gpu)} vs {len(ref)} windows"
    for k in ("baseline", "window_ap", "t_start"):
        assert np.array_equal(gpu[k], ref[k]), f"{label}: key {k} differs"
    n_amb = 0
    bad = []
    for i in range(len(ref)):
        g, r = gpu[i], ref[i]
        same_bin = (g["k_rate"], g["k_delay"]) == (r["k_rate"], r["k_delay"])
        if not same_bin:
            if r["margin"] >= RTOL:
                bad.append((i, "bin", (int(g["k_rate"]), int(g["k_delay"])),
                            (int(r["k_rate"]), int(r["k_delay"])), float(r["margin"])))
                continue
            n_amb += 1
            x = x_by_baseline(int(g["scan"]), int(g["baseline"]))
            p_here = oracle_power_at(x, int(r["t_start"]), int(r["window_ap"]), pad_freq,
                                     pad_time, int(g["k_rate"]), int(g["k_delay"]))
            p_max = float(r["amp"]) ** 2
            if p_here < p_max * (1 - RTOL):
                bad.append((i, "ambiguous-bin", p_here, p_max))
                continue
        for k in ("amp", "snr", "energy"):
            gv, rv = float(g[k]), float(r[k])
            if not math.isclose(gv, rv, rel_tol=RTOL, abs_tol=1e-6):
                bad.append((i, k, gv, rv))
        if same_bin:
            for k in ("delay_s", "rate_hz"):
                if not math.isclose(float(g[k]), float(r[k]), rel_tol=1e-9, abs_tol=1e-300):
                    bad.append((i, k, float(g[k]), float(r[k])))
    assert not bad, f"{label}: {len(bad)} mismatches, first: {bad[:5]}"
    return n_amb


def compare_candidates(gpu_c, ref_table, threshold, label=""):
    """Candidate keys must equal the reference's, up to windows whose
    reference SNR is within 1e-4 relative of the threshold."""
    def keys(a):
        return [(int(r["scan"]), int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))
                for r in a]
    gk = keys(gpu_c)
    assert gk == sorted(gk), f"{label}: candidates not in key order"
    ref_c = ref_table[ref_table["snr"] > threshold]
    rk = keys(ref_c)
    near = set(keys(ref_table[np.abs(ref_table["snr"] - threshold) < RTOL * max(threshold, 1e-30)]))
    diff = set(gk) ^ set(rk)
    assert diff <= near, f"{label}: candidate lists differ at {sorted(diff - near)[:10]}"


def oracle_table(scans_vis, scans, window_aps, pad_freq, pad_time, threshold, delay_only=False,
                 gains=None, shifts=None):
    """Reference table for several scans, in window-id order, with `scan` set.
    gains: None, or per scan None / a (B, F) array of calibration gains;
    shifts: None, or per scan None / an (F,) array of dedispersion shifts."""
    tabs = []
    for s, (v, d) in enumerate(zip(scans_vis, scans)):
        g = None if gains is None else gains[s]
        sh = None if shifts is None else shifts[s]
        t, _ = fo.search_scan(v, window_aps, pad_freq, pad_time, threshold, d["ap_seconds"],
                              d["chan_width_hz"], scan=s, delay_only=delay_only, gains=g,
                              shifts=sh)
        tabs.append(t)
    return np.concatenate(tabs)
