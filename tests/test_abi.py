"""CPU-only checks of the C ABI: the library loads, exports every entry
point declared in include/*.h, and its host-side validation and
sizing behave as documented (no device work is done here)."""

import ctypes
import os
import re

import numpy as np

import pytest

import paper_2108_05602_amd as F
from paper_2108_05602_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C2 = dict(n_baselines=45, n_ap=58600, n_if=8, n_chan=32, ap_seconds=1.024e-3,
          chan_width_hz=0.5e6)
C2_W = [1, 2, 4, 8, 16, 32]


def declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc))
                   if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = F.load()
    decl = declared_functions()
    assert set(decl) == set(B.ENTRY_POINTS), decl
    for name in decl:
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_struct_layouts():
    assert ctypes.sizeof(B.fringe_scan_desc) == 32
    assert ctypes.sizeof(B.fringe_params) == 48
    assert ctypes.sizeof(B.fringe_candidate) == 56
    assert ctypes.sizeof(B.fringe_plan_summary) == 32
    assert ctypes.sizeof(B.fringe_match_params) == 8
    assert B.PULSE_DTYPE.itemsize == 72
    assert ctypes.sizeof(B.fringe_serve_result) == 64


def test_monotonic_clock_is_perf_counter():
    """The server's timestamps share time.perf_counter's clock."""
    import time
    for _ in range(3):
        a = time.perf_counter()
        b = B.fringe_monotonic_ns() * 1e-9
        c = time.perf_counter()
        assert a - 1e-3 <= b <= c + 1e-3


def test_server_argument_checks():
    """Refused on the host, before any device work."""
    lib = F.load()
    out = ctypes.c_void_p()
    sa = B._scan_array([C2])
    p, keep = B._params(C2_W, 4, 2, 4.5, 0, 1024, 0)
    assert lib.fringe_server_create(None, 1, ctypes.byref(p), 0, 0, ctypes.byref(out)) == B.FRINGE_E_INVALID
    assert lib.fringe_server_create(sa, 0, ctypes.byref(p), 0, 0, ctypes.byref(out)) == B.FRINGE_E_INVALID
    assert lib.fringe_server_create(sa, 1, ctypes.byref(p), 0, 2, ctypes.byref(out)) == B.FRINGE_E_INVALID
    assert lib.fringe_server_create(sa, 1, ctypes.byref(p), 0, 0, None) == B.FRINGE_E_INVALID
    for flag in (B.FRINGE_PLAIN, B.FRINGE_GRAPH):
        q, keep2 = B._params(C2_W, 4, 2, 4.5, 0, 1024, flag)
        assert lib.fringe_server_create(sa, 1, ctypes.byref(q), 0, 0,
                                        ctypes.byref(out)) == B.FRINGE_E_UNSUPPORTED
    n = ctypes.c_int64()
    n32 = ctypes.c_int32()
    assert lib.fringe_server_submit(None, 0, 0, ctypes.c_void_p(0x1000)) == B.FRINGE_E_INVALID
    assert lib.fringe_server_poll(None, None, 0, ctypes.byref(n32), None, 0,
                                  ctypes.byref(n)) == B.FRINGE_E_INVALID
    assert lib.fringe_server_pending(None, ctypes.byref(n)) == B.FRINGE_E_INVALID
    assert lib.fringe_server_set_shifts(None, 0, None) == B.FRINGE_E_INVALID
    assert lib.fringe_server_destroy(None) == B.FRINGE_E_INVALID


def test_dedisperse_argument_checks():
    # host-side validation only: rejected before any launch
    for args in [(0, 4096, 1, 10, 8, 64), (64, 0, 1, 10, 8, 64), (64, 4096, 0, 10, 8, 64),
                 (64, 4096, 1, 0, 8, 64), (64, 4096, 1, 10, 8, 0)]:
        with pytest.raises(F.FringeError) as e:
            F.fringe_dedisperse(*args)
        assert e.value.code == B.FRINGE_E_INVALID
    # overlapping input and output (1 x 10 x 8 samples of 8 bytes = 640 bytes)
    with pytest.raises(F.FringeError) as e:
        F.fringe_dedisperse(4096, 4096 + 320, 1, 10, 8, 64)
    assert "overlap" in str(e.value)


def test_probe_argument_checks():
    # host-side validation only: every call below is rejected before a launch
    with pytest.raises(F.FringeError):
        B.fringe_probe_fma(0, 10, 16)
    with pytest.raises(F.FringeError):
        B.fringe_probe_fma(1, 0, 16)
    with pytest.raises(F.FringeError):
        B.fringe_probe_fma(1, 10, 0)
    with pytest.raises(F.FringeError):
        B.fringe_probe_copy(16, 32, 15)
    with pytest.raises(F.FringeError):
        B.fringe_probe_copy(16, 40, 64)
    with pytest.raises(F.FringeError):
        B.fringe_probe_copy(0, 32, 64)


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert F.fringe_strerror(code)
    assert F.fringe_strerror(-99) == "unknown error"


def test_window_counts_match_closed_form():
    s = F.fringe_plan_check([C2], C2_W, snr_threshold=4.5)
    assert s["n_windows"] == 7745940
    assert s["max_window_ap"] == 32
    c5 = dict(n_baselines=66, n_ap=117200, n_if=16, n_chan=64, ap_seconds=0.512e-3,
              chan_width_hz=0.25e6)
    s5 = F.fringe_plan_check([c5], [1, 2, 4, 8, 16, 32, 64, 128], snr_threshold=4.5)
    assert s5["n_windows"] == 23084226
    c1 = dict(n_baselines=1, n_ap=64, n_if=2, n_chan=16, ap_seconds=1.0, chan_width_hz=1 / 32)
    assert F.fringe_plan_check([c1], [4], snr_threshold=3.0)["n_windows"] == 31
    # several scans add up; a scan shorter than every window has none
    short = dict(c1, n_ap=3)
    assert F.fringe_plan_check([c1, short, c1], [4], snr_threshold=3.0)["n_windows"] == 62


def _code(fn):
    with pytest.raises(F.FringeError) as e:
        fn()
    return e.value.code


def test_validation_errors():
    ok = dict(n_baselines=2, n_ap=100, n_if=4, n_chan=16, ap_seconds=1e-3, chan_width_hz=1e6)
    chk = F.fringe_plan_check
    assert _code(lambda: chk([dict(ok, n_chan=12)], [4])) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: chk([dict(ok, n_baselines=0)], [4])) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([dict(ok, ap_seconds=0.0)], [4])) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [3])) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: chk([ok], [256])) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: chk([ok], [4, 2])) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [4, 4])) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [])) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [4], pad_freq=3)) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: chk([ok], [4], pad_time=4)) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: chk([ok], [4], snr_threshold=-1.0)) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [4], snr_threshold=float("nan"))) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [4], max_candidates=-1)) == B.FRINGE_E_INVALID
    assert _code(lambda: chk([ok], [4], flags=0x80)) == B.FRINGE_E_INVALID
    # M_f = pad * F must lie in [64, 4096]
    assert _code(lambda: chk([dict(ok, n_if=1, n_chan=8)], [4], pad_freq=4)) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: chk([dict(ok, n_if=16, n_chan=128)], [4], pad_freq=4)) == B.FRINGE_E_UNSUPPORTED
    assert "power of two" in F.fringe_last_error() or F.fringe_last_error()
    # a baseline of 4 GiB or more of samples: not with windows of at most 64
    # APs (the fused kernel's 32-bit offsets serve them, also in plans that
    # have longer windows); windows longer than 64 APs alone are fine
    big = dict(ok, n_baselines=1, n_ap=600000, n_if=16, n_chan=64)
    assert _code(lambda: chk([big], [64, 128])) == B.FRINGE_E_UNSUPPORTED
    assert "4 GiB" in F.fringe_last_error()
    assert chk([big], [128])["n_windows"] > 0
    # the fused kernel folds at most 16 x 64 channels per lane: wider bands
    # (M_f = 4096 at pad 2 or 1) only with windows longer than 64 APs
    wide = dict(ok, n_if=32, n_chan=64)
    assert _code(lambda: chk([wide], [4], pad_freq=2)) == B.FRINGE_E_UNSUPPORTED
    assert "16 x 64" in F.fringe_last_error() or "<= 1024" in F.fringe_last_error()
    assert _code(lambda: chk([dict(wide, n_if=64)], [1, 2], pad_freq=1)) == B.FRINGE_E_UNSUPPORTED
    assert chk([dict(wide, n_ap=300)], [128], pad_freq=2)["n_windows"] > 0


def test_budget():
    s = F.fringe_plan_check([C2], C2_W, snr_threshold=4.5)
    # a budget that does not hold every baseline's work buffers at once is
    # met by processing the baselines in slabs
    budget = 300 << 20
    b = F.fringe_plan_check([C2], C2_W, snr_threshold=4.5, hbm_budget_bytes=budget)
    assert b["device_bytes"] <= budget
    assert 1 <= b["slab_baselines"] < s["slab_baselines"] == 45
    # windows longer than 32 APs take the two-pass path, whose delay spectra
    # (8 bytes per delay bin per AP) dominate the work buffers
    c5 = dict(n_baselines=66, n_ap=117200, n_if=16, n_chan=64, ap_seconds=0.512e-3,
              chan_width_hz=0.25e6)
    s5 = F.fringe_plan_check([c5], [1, 2, 4, 8, 16, 32, 64, 128], snr_threshold=4.5)
    assert s5["scratch_bytes"] >= s5["slab_baselines"] * 117200 * 4096 * 8
    # below the result buffers themselves: refused
    assert _code(lambda: F.fringe_plan_check([C2], C2_W, hbm_budget_bytes=1 << 20)) == B.FRINGE_E_NOMEM


def test_plain_flag_rules():
    c1 = dict(n_baselines=1, n_ap=64, n_if=2, n_chan=16, ap_seconds=1.0, chan_width_hz=1 / 32)
    assert F.fringe_plan_check([c1], [4], flags=B.FRINGE_PLAIN)["n_windows"] == 31
    assert _code(lambda: F.fringe_plan_check([dict(c1, n_ap=256)], [128], flags=B.FRINGE_PLAIN)) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: F.fringe_plan_check([c1], [4], flags=B.FRINGE_PLAIN | B.FRINGE_STREAMING)) == B.FRINGE_E_INVALID


def test_graph_flag_rules():
    """FRINGE_GRAPH is for batch plans: not with streaming, profiling or the
    one-window-per-launch path."""
    c1 = dict(n_baselines=1, n_ap=64, n_if=2, n_chan=16, ap_seconds=1.0, chan_width_hz=1 / 32)
    assert F.fringe_plan_check([c1], [4], flags=B.FRINGE_GRAPH)["n_windows"] == 31
    assert F.fringe_plan_check([c1], [4], flags=B.FRINGE_GRAPH | B.FRINGE_DUMP_GRID)["n_windows"] == 31
    for other in (B.FRINGE_STREAMING, B.FRINGE_PROFILE, B.FRINGE_PLAIN):
        assert _code(lambda: F.fringe_plan_check([c1], [4], flags=B.FRINGE_GRAPH | other)) == B.FRINGE_E_INVALID
    assert _code(lambda: F.fringe_plan_check([c1], [4], flags=0x80)) == B.FRINGE_E_INVALID
    assert F.fringe_plan_check([c1], [4], flags=B.FRINGE_AUTOTUNE)["n_windows"] == 31


def test_delay_only_flag_rules():
    """FRINGE_DELAY_ONLY: same windows, windows of at most 64 APs, no grid
    dump.  Its work buffers hold per window and wave a peak key (8 B) and a
    power sum (4 B): on bands of up to 256 channels a wave takes four of the
    M_f / 64 delay-bin classes (4 waves for the 16 classes at 256 channels,
    against the full search's 16 keys of 8 B), on wider bands two (16 waves
    for the 32 classes at 512 channels, against 32 keys)."""
    c1 = dict(n_baselines=1, n_ap=64, n_if=2, n_chan=16, ap_seconds=1.0, chan_width_hz=1 / 32)
    assert F.fringe_plan_check([c1], [4], flags=B.FRINGE_DELAY_ONLY)["n_windows"] == 31
    for flags in (B.FRINGE_DELAY_ONLY | B.FRINGE_STREAMING, B.FRINGE_DELAY_ONLY | B.FRINGE_PLAIN,
                  B.FRINGE_DELAY_ONLY | B.FRINGE_GRAPH):
        assert F.fringe_plan_check([c1], [1, 2, 4], flags=flags)["n_windows"] > 0
    assert _code(lambda: F.fringe_plan_check([dict(c1, n_ap=256)], [128],
                                             flags=B.FRINGE_DELAY_ONLY)) == B.FRINGE_E_UNSUPPORTED
    assert _code(lambda: F.fringe_plan_check([c1], [4], flags=B.FRINGE_DELAY_ONLY | B.FRINGE_DUMP_GRID)) == B.FRINGE_E_INVALID
    full = F.fringe_plan_check([C2], C2_W)
    do = F.fringe_plan_check([C2], C2_W, flags=B.FRINGE_DELAY_ONLY)
    assert do["n_windows"] == full["n_windows"]
    assert full["scratch_bytes"] - do["scratch_bytes"] == full["n_windows"] * (16 * 8 - 4 * 12)
    wide = dict(C2, n_if=16, n_ap=4096)
    full = F.fringe_plan_check([wide], C2_W)
    do = F.fringe_plan_check([wide], C2_W, flags=B.FRINGE_DELAY_ONLY)
    assert full["scratch_bytes"] - do["scratch_bytes"] == full["n_windows"] * (32 * 8 - 16 * 12)
    # 16 channels at pad 4: one class (M_f = 64) in a wave of four, the
    # other three ghosts: one key and sum per window against one key
    narrow = dict(C2, n_if=2, n_chan=8, n_ap=4096)
    full = F.fringe_plan_check([narrow], C2_W)
    do = F.fringe_plan_check([narrow], C2_W, flags=B.FRINGE_DELAY_ONLY)
    assert do["scratch_bytes"] - full["scratch_bytes"] == full["n_windows"] * 4


def test_streaming_sizing():
    # a 976-AP chunk of a 12-station subarray: windows ending in the chunk
    sub = dict(n_baselines=66, n_ap=976, n_if=8, n_chan=32, ap_seconds=1.024e-3, chan_width_hz=0.5e6)
    s = F.fringe_plan_check([sub], C2_W, flags=B.FRINGE_STREAMING)
    # at most floor((C - 1) / stride) + 1 windows of each length end in a chunk of C APs
    per_bl = sum((976 - 1) // max(1, w // 2) + 1 for w in C2_W)
    assert s["n_windows"] == 66 * per_bl
    assert _code(lambda: F.fringe_plan_check([sub], C2_W, flags=B.FRINGE_STREAMING | B.FRINGE_DUMP_GRID)) == B.FRINGE_E_INVALID


def test_dump_grid_only_for_small_plans():
    assert _code(lambda: F.fringe_plan_check([C2], C2_W, flags=B.FRINGE_DUMP_GRID)) == B.FRINGE_E_INVALID


def test_dm_shifts():
    """Dispersion shifts: the cold-plasma law at two frequencies, rounding to
    APs, the highest channel as the zero reference."""
    from paper_2108_05602_amd.dedisp import channel_freqs_hz, dm_shifts
    f = channel_freqs_hz(1.6e9, 8, 32, 0.5e6)
    assert f.shape == (256,) and f[0] == 1.6e9 and f[32] == 1.616e9 and f[-1] == 1.6e9 + 127.5e6
    d = dm_shifts(100.0, f, 1.024e-3)
    # 100 pc cm^-3 between 1600 and 1727.5 MHz: 4148.808 * 100 * (1600^-2 - 1727.5^-2) s
    want = 4148.808 * 100 * (1600.0 ** -2 - 1727.5 ** -2) / 1.024e-3
    assert d[0] == int(round(want)) and d[-1] == 0
    assert np.all(np.diff(d) <= 0) and d.dtype == np.int32
    assert np.all(dm_shifts(0.0, f, 1e-3) == 0)


def test_autospectrum_gains_argument_checks():
    """Refused on the host, before any device work."""
    g = F.fringe_autospectrum_gains
    assert _code(lambda: g(0, 3, 2, 64, 0x1000, 3, 0, 0x2000)) == B.FRINGE_E_INVALID
    assert _code(lambda: g(0x1000, 0, 2, 64, 0x2000, 3, 0, 0x3000)) == B.FRINGE_E_INVALID
    assert _code(lambda: g(0x1000, 3, 2, 64, 0x2000, 0, 0, 0x3000)) == B.FRINGE_E_INVALID
    # gains_in overlapping gains_out without being the same array
    assert _code(lambda: g(0x1000, 3, 2, 64, 0x2000, 3, 0x100000, 0x100008)) == B.FRINGE_E_INVALID
    assert "overlap" in F.fringe_last_error()


def test_tune_table_file_round_trip(tmp_path):
    """The tune table's JSON form: a written table loads back unchanged,
    entries merge by class, malformed files are refused and leave the
    table as it was (host code only, no device)."""
    import json
    src = tmp_path / "in.json"
    entries = [
        dict(arch="gfx950", cus=256, n_freq=1024, pad_freq=4, pad_time=2, log2_wmax=6,
             spectra=1, chunk=256, ms_fused=12.5, ms_spectra=10.25),
        dict(arch="gfx950", cus=256, n_freq=256, pad_freq=4, pad_time=0, log2_wmax=5,
             spectra=0, chunk=1024, ms_fused=3.0, ms_spectra=-1),
    ]
    src.write_text(json.dumps({"fringe_tune_table": 1, "entries": entries}, indent=1))
    F.fringe_tune_clear()
    F.fringe_tune_load(str(src))
    out = tmp_path / "out.json"
    F.fringe_tune_save(str(out))
    got = json.loads(out.read_text())
    assert got["fringe_tune_table"] == 1
    assert got["entries"] == entries
    # a later entry of the same class replaces the earlier one
    e2 = dict(entries[0], chunk=512, spectra=0)
    src.write_text(json.dumps({"fringe_tune_table": 1, "entries": [e2]}))
    F.fringe_tune_load(str(src))
    F.fringe_tune_save(str(out))
    got = json.loads(out.read_text())["entries"]
    assert len(got) == 2 and got[0] == e2
    for bad in ('{"entries": []}', '{"fringe_tune_table": 1, "entries": [{"arch": 3}]}',
                '{"fringe_tune_table": 1, "entries": [{"arch": "gfx950", "cus": 1}]}',
                '{"fringe_tune_table": 1, "entries": [', 'not json'):
        src.write_text(bad)
        assert _code(lambda: F.fringe_tune_load(str(src))) == B.FRINGE_E_INVALID
    F.fringe_tune_save(str(out))
    assert len(json.loads(out.read_text())["entries"]) == 2
    assert _code(lambda: F.fringe_tune_load(str(tmp_path / "missing.json"))) == B.FRINGE_E_INVALID
    F.fringe_tune_clear()
    F.fringe_tune_save(str(out))
    assert json.loads(out.read_text())["entries"] == []


def test_shipped_tune_table_loads():
    """The tune table shipped for MI355X (written by the autotuner there)
    loads and covers the batched workload's four band classes."""
    import json
    path = os.path.join(ROOT, "paper_2108_05602_amd", "tune", "gfx950_256cu.json")
    data = json.load(open(path))
    assert data["fringe_tune_table"] == 1
    got = sorted(e["n_freq"] for e in data["entries"])
    assert got == [128, 256, 512, 1024]
    for e in data["entries"]:
        assert e["arch"] == "gfx950" and e["cus"] == 256 and e["chunk"] in (128, 256, 512, 1024)
        assert e["spectra"] in (0, 1) and e["pad_freq"] == 4 and e["pad_time"] == 2
    F.fringe_tune_clear()
    F.fringe_tune_load(path)
    F.fringe_tune_clear()


def test_chunk_argument_checks():
    """fringe_plan_set_chunk / _get_chunk refuse a null plan or output on
    the host (the rules that need a plan run on the GPU)."""
    lib = F.load()
    out = ctypes.c_int32()
    assert lib.fringe_plan_set_chunk(None, 0, 256) == B.FRINGE_E_INVALID
    assert lib.fringe_plan_get_chunk(None, 0, ctypes.byref(out)) == B.FRINGE_E_INVALID
