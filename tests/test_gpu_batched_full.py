"""The batched uneven workload at its full recipe (200 scans of 10-120 s,
3-66 baselines, 8 or 16 IF x 16/32/64 channels, windows 1-64 APs: about
1.1 G windows over 1.3 TB), generated on the device in waves that fit HBM;
each wave is one plan (one fused launch per fold class of its bands).

Every wave is checked against the CPU reference on samples, the windows'
APs copied back to the host: 40 random windows, 40 drawn from those within
1 % of the threshold (found by a second search of the wave at 0.99 x
threshold), 30 from above that band; and by properties of its whole
candidate list (in key order, each record equal to the low-threshold
search's, every window of that search above 1.01 x threshold in it, none
at or below the threshold)."""

import numpy as np
import pytest

import oracle.fringe_oracle as fo
import synth
from fringe_testlib import compare_windows

pytestmark = pytest.mark.gpu

WAVE_BYTES = 150_000_000_000


class _DeviceBaseline:
    """One baseline of a device cube; slicing copies those APs to the host."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, sl):
        seg = self.t[sl]
        return seg.reshape(seg.shape[0], -1).cpu().numpy()


def _ref_rows(rows, specs, idx, tens, p):
    out = []
    for g in rows:
        s = int(g["scan"])
        sp = specs[idx[s]]
        w, t0, b = int(g["window_ap"]), int(g["t_start"]), int(g["baseline"])
        seg = _DeviceBaseline(tens[s][b])[t0:t0 + w]
        r = fo.search_window(seg, 0, w, p["pad_freq"], p["pad_time"])
        m_f, m_t = p["pad_freq"] * sp.n_freq, p["pad_time"] * w
        out.append((s, b, w, t0, r.k_rate, r.k_delay, r.amp, r.snr, r.energy,
                    fo.signed_bin(r.k_delay, m_f) / (m_f * sp.chan_width_hz),
                    fo.signed_bin(r.k_rate, m_t) / (m_t * sp.ap_seconds), r.margin))
    return np.array(out, dtype=fo.TABLE_DTYPE)


def test_batched_uneven_full_recipe():
    import torch

    import paper_2108_05602_amd as F
    from synth import device as sd
    specs = synth.c3()
    p = synth.C3_PARAMS
    thr = p["snr_threshold"]
    groups = sd.waves(specs, WAVE_BYTES)
    print(f"case: batched uneven full recipe, {len(specs)} scans, "
          f"{sum(s.nbytes() for s in specs) / 1e12:.2f} TB in {len(groups)} waves", flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    common = dict(pad_freq=p["pad_freq"], pad_time=p["pad_time"], max_candidates=1 << 23)
    rng = np.random.default_rng(303)
    total = 0
    for wi, idx in enumerate(groups):
        tens = [sd.generate(specs[i]) for i in idx]
        descs = [specs[i].desc() for i in idx]
        ptrs = [t.data_ptr() for t in tens]
        with F.Plan(descs, p["window_aps"], snr_threshold=thr, flags=F.FRINGE_PROFILE,
                    **common) as plan:
            plan.search(ptrs, stream)
            cands = plan.candidates()
            n_win = plan.info()["n_windows"]
            launches = plan.profile()["rate_launches"]
            srows = plan.windows(np.sort(rng.choice(n_win, 40, replace=False)))
        want = sum(sum(n for n in [((specs[i].n_ap - w) // max(1, w // 2) + 1)
                                   for w in p["window_aps"]]) * specs[i].n_baselines for i in idx)
        assert n_win == want
        total += n_win
        with F.Plan(descs, p["window_aps"], snr_threshold=0.99 * thr, **common) as low:
            low.search(ptrs, stream)
            above = low.candidates()
        band = above[above["snr"] <= 1.01 * thr]
        high = above[above["snr"] > 1.01 * thr]
        print(f"wave {wi}: {len(idx)} scans, {n_win} windows, {launches} fused launches, "
              f"{len(cands)} candidates, {len(band)} in the 1 % band", flush=True)

        def xb(s, b):
            return _DeviceBaseline(tens[s][b])

        compare_windows(srows, _ref_rows(srows, specs, idx, tens, p), xb, p["pad_freq"],
                        p["pad_time"], f"wave {wi} sample")
        pb = band[np.sort(rng.choice(len(band), min(40, len(band)), replace=False))]
        compare_windows(pb, _ref_rows(pb, specs, idx, tens, p), xb, p["pad_freq"],
                        p["pad_time"], f"wave {wi} band")
        ph = high[np.sort(rng.choice(len(high), min(30, len(high)), replace=False))]
        ref_h = _ref_rows(ph, specs, idx, tens, p)
        compare_windows(ph, ref_h, xb, p["pad_freq"], p["pad_time"], f"wave {wi} high")
        assert np.all(ref_h["snr"] > thr)

        def key(r):
            return (int(r["scan"]), int(r["baseline"]), int(r["window_ap"]), int(r["t_start"]))
        got = [key(c) for c in cands]
        assert got == sorted(got)
        low_by_key = {key(r): r for r in above}
        for c in cands:
            r = low_by_key[key(c)]
            assert (r["k_rate"], r["k_delay"], r["amp"], r["snr"]) == \
                (c["k_rate"], c["k_delay"], c["amp"], c["snr"])
        assert {key(r) for r in high} <= set(got)
        assert np.all(cands["snr"] > thr)
        del tens
        torch.cuda.empty_cache()
    print(f"{total} windows checked over {len(groups)} waves", flush=True)
    assert total > 1_000_000_000
