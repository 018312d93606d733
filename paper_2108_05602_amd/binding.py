"""ctypes binding of libfringe (include/fringe.h, include/fringe_calib.h,
include/fringe_match.h, include/fringe_probe.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
computation of its own; all search work runs in the library's HIP kernels,
the matching and localization of candidates in its host code.
Device buffers are passed as integer addresses (e.g. torch.Tensor.data_ptr())
and streams as integer hipStream_t handles (torch.cuda.Stream.cuda_stream).
The library must have been built (python -m paper_2108_05602_amd.build);
loading fails loudly otherwise.  In a process that also uses torch, import
torch first: the library then binds to the HIP runtime torch has loaded
(loaded first, it would bring a second runtime that sees no device).
"""

from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_float, c_int, c_int32,
                    c_int64, c_uint32, c_uint64, c_void_p)
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libfringe.so")

FRINGE_OK = 0
FRINGE_E_INVALID = -1
FRINGE_E_UNSUPPORTED = -2
FRINGE_E_NOMEM = -3
FRINGE_E_HIP = -4
FRINGE_E_CAPACITY = -5
FRINGE_E_STATE = -6

FRINGE_STREAMING = 0x1
FRINGE_DUMP_GRID = 0x2
FRINGE_PROFILE = 0x4
FRINGE_PLAIN = 0x8
FRINGE_GRAPH = 0x10
FRINGE_DELAY_ONLY = 0x20
FRINGE_AUTOTUNE = 0x40

ENTRY_POINTS = (
    "fringe_plan_check", "fringe_plan", "fringe_search", "candidates_get",
    "fringe_windows_get", "fringe_window_id", "fringe_grid_get", "fringe_profile_get",
    "fringe_plan_info", "fringe_set_gains", "fringe_set_shifts", "fringe_dedisperse",
    "fringe_plan_destroy", "fringe_strerror", "fringe_last_error",
    "fringe_match", "fringe_localize", "fringe_delay_partials",
    "fringe_probe_fma", "fringe_probe_copy", "fringe_search_noalloc",
    "fringe_autospectrum_gains", "fringe_tune_load", "fringe_tune_save", "fringe_tune_clear",
    "fringe_plan_tuning", "fringe_plan_set_chunk", "fringe_plan_get_chunk",
    "fringe_monotonic_ns", "fringe_server_create", "fringe_server_set_shifts",
    "fringe_server_submit", "fringe_server_poll", "fringe_server_pending",
    "fringe_server_destroy",
)


class fringe_serve_result(Structure):
    _fields_ = [("sub", c_int32), ("status", c_int32), ("tag", c_int64),
                ("n_candidates", c_int64), ("n_total", c_int64), ("n_windows", c_int64),
                ("t_submit_ns", c_int64), ("t_launch_ns", c_int64), ("t_done_ns", c_int64)]


class fringe_scan_desc(Structure):
    _fields_ = [("n_baselines", c_int32), ("n_ap", c_int32), ("n_if", c_int32),
                ("n_chan", c_int32), ("ap_seconds", c_double), ("chan_width_hz", c_double)]


class fringe_params(Structure):
    _fields_ = [("window_aps", POINTER(c_int32)), ("n_window_lengths", c_int32),
                ("pad_freq", c_int32), ("pad_time", c_int32), ("snr_threshold", c_float),
                ("hbm_budget_bytes", c_uint64), ("max_candidates", c_int64),
                ("flags", c_uint32)]


class fringe_candidate(Structure):
    _fields_ = [("scan", c_int32), ("baseline", c_int32), ("window_ap", c_int32),
                ("t_start", c_int32), ("k_rate", c_int32), ("k_delay", c_int32),
                ("amp", c_float), ("snr", c_float), ("energy", c_float),
                ("reserved", c_int32), ("delay_s", c_double), ("rate_hz", c_double)]


class fringe_plan_summary(Structure):
    _fields_ = [("n_windows", c_int64), ("device_bytes", c_int64), ("scratch_bytes", c_int64),
                ("max_window_ap", c_int32), ("slab_baselines", c_int32)]


class fringe_tune_entry(Structure):
    _fields_ = [("n_freq", c_int32), ("pad_freq", c_int32), ("pad_time", c_int32),
                ("log2_wmax", c_int32), ("spectra", c_int32), ("chunk", c_int32),
                ("ms_fused", c_float), ("ms_spectra", c_float)]


class fringe_profile(Structure):
    _fields_ = [("delay_ms", c_double), ("rate_ms", c_double), ("finalize_ms", c_double),
                ("compact_ms", c_double), ("delay_launches", c_int32),
                ("rate_launches", c_int32), ("finalize_launches", c_int32),
                ("compact_launches", c_int32)]


CANDIDATE_DTYPE = np.dtype([
    ("scan", np.int32), ("baseline", np.int32), ("window_ap", np.int32),
    ("t_start", np.int32), ("k_rate", np.int32), ("k_delay", np.int32),
    ("amp", np.float32), ("snr", np.float32), ("energy", np.float32),
    ("reserved", np.int32), ("delay_s", np.float64), ("rate_hz", np.float64),
], align=True)
assert CANDIDATE_DTYPE.itemsize == ctypes.sizeof(fringe_candidate) == 56


class fringe_match_params(Structure):
    _fields_ = [("min_windows", c_int32), ("min_baselines", c_int32)]


PULSE_DTYPE = np.dtype([
    ("scan", np.int32), ("pulse", np.int32), ("baseline", np.int32), ("window_ap", np.int32),
    ("t_start", np.int32), ("k_rate", np.int32), ("k_delay", np.int32), ("t_lo", np.int32),
    ("t_hi", np.int32), ("n_windows", np.int32), ("n_lengths", np.int32),
    ("amp", np.float32), ("snr", np.float32), ("reserved", np.int32),
    ("delay_s", np.float64), ("rate_hz", np.float64),
], align=True)
assert PULSE_DTYPE.itemsize == 72


class FringeError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__(f"{where}: {fringe_strerror(code)} ({code}): {detail}")


_lib = None


def load(path: Optional[str] = None):
    """Load libfringe.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2108_05602_amd.build`")
    lib = ctypes.CDLL(path)
    lib.fringe_plan_check.argtypes = [POINTER(fringe_scan_desc), c_int32, POINTER(fringe_params),
                                      POINTER(fringe_plan_summary)]
    lib.fringe_plan.argtypes = [POINTER(fringe_scan_desc), c_int32, POINTER(fringe_params),
                                POINTER(c_void_p)]
    lib.fringe_search.argtypes = [c_void_p, POINTER(c_void_p), c_void_p]
    lib.candidates_get.argtypes = [c_void_p, c_void_p, c_int64, POINTER(c_int64)]
    lib.fringe_windows_get.argtypes = [c_void_p, POINTER(c_int64), c_int64, c_void_p]
    lib.fringe_window_id.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, POINTER(c_int64)]
    lib.fringe_grid_get.argtypes = [c_void_p, c_int64, c_void_p, c_int64]
    lib.fringe_plan_info.argtypes = [c_void_p, POINTER(fringe_plan_summary)]
    lib.fringe_profile_get.argtypes = [c_void_p, POINTER(fringe_profile)]
    lib.fringe_plan_destroy.argtypes = [c_void_p]
    lib.fringe_plan_destroy.restype = None
    lib.fringe_strerror.argtypes = [c_int]
    lib.fringe_strerror.restype = c_char_p
    lib.fringe_last_error.argtypes = []
    lib.fringe_last_error.restype = c_char_p
    lib.fringe_match.argtypes = [c_void_p, c_int64, POINTER(fringe_match_params), c_void_p,
                                 c_int64, POINTER(c_int64), POINTER(c_int64)]
    dp = POINTER(c_double)
    lib.fringe_localize.argtypes = [dp, dp, dp, c_int32, dp, dp, dp, dp]
    lib.fringe_delay_partials.argtypes = [dp, c_int32, c_double, c_double, c_double, dp, dp]
    lib.fringe_dedisperse.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                      c_void_p]
    lib.fringe_probe_fma.argtypes = [c_int64, c_int32, c_void_p, dp, c_void_p]
    lib.fringe_probe_copy.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
    lib.fringe_search_noalloc.argtypes = [POINTER(fringe_scan_desc), POINTER(fringe_params),
                                          c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
    lib.fringe_autospectrum_gains.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                              c_int32, c_void_p, c_void_p, c_void_p]
    lib.fringe_tune_load.argtypes = [c_char_p]
    lib.fringe_tune_save.argtypes = [c_char_p]
    lib.fringe_tune_clear.argtypes = []
    lib.fringe_tune_clear.restype = None
    lib.fringe_plan_tuning.argtypes = [c_void_p, POINTER(fringe_tune_entry), c_int32,
                                       POINTER(c_int32)]
    lib.fringe_monotonic_ns.argtypes = []
    lib.fringe_monotonic_ns.restype = c_int64
    lib.fringe_server_create.argtypes = [POINTER(fringe_scan_desc), c_int32, POINTER(fringe_params),
                                         c_int32, c_int32, POINTER(c_void_p)]
    lib.fringe_server_set_shifts.argtypes = [c_void_p, c_int32, c_void_p]
    lib.fringe_server_submit.argtypes = [c_void_p, c_int32, c_int64, c_void_p]
    lib.fringe_server_poll.argtypes = [c_void_p, POINTER(fringe_serve_result), c_int32,
                                       POINTER(c_int32), c_void_p, c_int64, POINTER(c_int64)]
    lib.fringe_server_pending.argtypes = [c_void_p, POINTER(c_int64)]
    lib.fringe_server_destroy.argtypes = [c_void_p]
    lib.fringe_plan_set_chunk.argtypes = [c_void_p, c_int32, c_int32]
    lib.fringe_plan_get_chunk.argtypes = [c_void_p, c_int32, POINTER(c_int32)]
    for name in ENTRY_POINTS:
        if name not in ("fringe_plan_destroy", "fringe_strerror", "fringe_last_error",
                        "fringe_tune_clear", "fringe_monotonic_ns"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def fringe_strerror(code: int) -> str:
    return load().fringe_strerror(code).decode()


def fringe_last_error() -> str:
    return load().fringe_last_error().decode()


def _check(rc: int, where: str):
    if rc != FRINGE_OK:
        raise FringeError(rc, where, fringe_last_error())


# ------------------------------------------------------------ marshalling --

def _scan_array(scans: Sequence[dict]):
    arr = (fringe_scan_desc * len(scans))()
    for i, s in enumerate(scans):
        arr[i] = fringe_scan_desc(int(s["n_baselines"]), int(s["n_ap"]), int(s["n_if"]),
                                  int(s["n_chan"]), float(s["ap_seconds"]),
                                  float(s["chan_width_hz"]))
    return arr


def _params(window_aps: Iterable[int], pad_freq: int, pad_time: int, snr_threshold: float,
            hbm_budget_bytes: int, max_candidates: int, flags: int):
    w = list(int(v) for v in window_aps)
    warr = (c_int32 * max(1, len(w)))(*w)
    p = fringe_params(ctypes.cast(warr, POINTER(c_int32)) if w else None, len(w), int(pad_freq),
                      int(pad_time), float(snr_threshold), int(hbm_budget_bytes),
                      int(max_candidates), int(flags))
    return p, warr


def fringe_plan_check(scans: Sequence[dict], window_aps, pad_freq=4, pad_time=2,
                      snr_threshold=4.5, hbm_budget_bytes=0, max_candidates=1 << 16,
                      flags=0) -> dict:
    """Validate and size without touching the GPU; raises FringeError."""
    lib = load()
    sa = _scan_array(scans)
    p, keep = _params(window_aps, pad_freq, pad_time, snr_threshold, hbm_budget_bytes,
                      max_candidates, flags)
    out = fringe_plan_summary()
    _check(lib.fringe_plan_check(sa, len(scans), ctypes.byref(p), ctypes.byref(out)),
           "fringe_plan_check")
    return {k: getattr(out, k) for k, _ in fringe_plan_summary._fields_}


def fringe_plan(scans: Sequence[dict], window_aps, pad_freq=4, pad_time=2, snr_threshold=4.5,
                hbm_budget_bytes=0, max_candidates=1 << 16, flags=0) -> int:
    """Create a plan on the current HIP device; returns its handle."""
    lib = load()
    sa = _scan_array(scans)
    p, keep = _params(window_aps, pad_freq, pad_time, snr_threshold, hbm_budget_bytes,
                      max_candidates, flags)
    h = c_void_p()
    _check(lib.fringe_plan(sa, len(scans), ctypes.byref(p), ctypes.byref(h)), "fringe_plan")
    return h.value


def fringe_search(plan: int, vis_ptrs: Sequence[Optional[int]], stream: int = 0) -> None:
    """Enqueue a search; vis_ptrs are device addresses (0/None = no chunk)."""
    lib = load()
    arr = (c_void_p * len(vis_ptrs))(*[int(v) if v else None for v in vis_ptrs])
    _check(lib.fringe_search(c_void_p(plan), arr, c_void_p(int(stream) if stream else None)),
           "fringe_search")


def candidates_get(plan: int, capacity: Optional[int] = None) -> np.ndarray:
    """All candidates of the last search, sorted (two-call pattern inside).
    Raises FringeError(FRINGE_E_CAPACITY) if they overflowed the plan's
    max_candidates."""
    lib = load()
    total = c_int64(0)
    if capacity is None:
        rc = lib.candidates_get(c_void_p(plan), None, 0, ctypes.byref(total))
        if rc not in (FRINGE_OK, FRINGE_E_CAPACITY):
            _check(rc, "candidates_get")
        capacity = total.value
    out = np.zeros(max(1, int(capacity)), dtype=CANDIDATE_DTYPE)
    rc = lib.candidates_get(c_void_p(plan), out.ctypes.data_as(c_void_p), int(capacity),
                            ctypes.byref(total))
    _check(rc, "candidates_get")
    return out[:min(int(capacity), total.value)]


def candidates_get_raw(plan: int, capacity: int, max_candidates: int):
    """(return code, n_total, copied records) without raising on
    FRINGE_E_CAPACITY; the library copies min(capacity, max_candidates,
    n_total) records."""
    lib = load()
    total = c_int64(0)
    out = np.zeros(max(1, int(capacity)), dtype=CANDIDATE_DTYPE)
    rc = lib.candidates_get(c_void_p(plan), out.ctypes.data_as(c_void_p), int(capacity),
                            ctypes.byref(total))
    n = max(0, min(int(capacity), int(max_candidates), total.value))
    return rc, total.value, out[:n]


def fringe_windows_get(plan: int, ids) -> np.ndarray:
    lib = load()
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int64))
    out = np.zeros(max(1, ids.size), dtype=CANDIDATE_DTYPE)
    _check(lib.fringe_windows_get(c_void_p(plan), ids.ctypes.data_as(POINTER(c_int64)),
                                  ids.size, out.ctypes.data_as(c_void_p)),
           "fringe_windows_get")
    return out[:ids.size]


def fringe_window_id(plan: int, scan: int, baseline: int, window_ap: int, t_start: int) -> int:
    lib = load()
    out = c_int64(0)
    _check(lib.fringe_window_id(c_void_p(plan), scan, baseline, window_ap, t_start,
                                ctypes.byref(out)), "fringe_window_id")
    return out.value


def fringe_grid_get(plan: int, window_id: int, m_t: int, m_f: int) -> np.ndarray:
    lib = load()
    out = np.zeros((m_t, m_f), dtype=np.complex64)
    _check(lib.fringe_grid_get(c_void_p(plan), int(window_id), out.ctypes.data_as(c_void_p),
                               out.size), "fringe_grid_get")
    return out


def fringe_profile_get(plan: int) -> dict:
    lib = load()
    out = fringe_profile()
    _check(lib.fringe_profile_get(c_void_p(plan), ctypes.byref(out)), "fringe_profile_get")
    return {k: getattr(out, k) for k, _ in fringe_profile._fields_}


def fringe_plan_info(plan: int) -> dict:
    lib = load()
    out = fringe_plan_summary()
    _check(lib.fringe_plan_info(c_void_p(plan), ctypes.byref(out)), "fringe_plan_info")
    return {k: getattr(out, k) for k, _ in fringe_plan_summary._fields_}


def fringe_set_gains(plan: int, scan: int, d_gains) -> None:
    """d_gains: device address (int) of [n_baselines][F] complex64 gains, or None."""
    lib = load()
    _check(lib.fringe_set_gains(c_void_p(plan), c_int32(int(scan)), c_void_p(d_gains or None)),
           "fringe_set_gains")


def fringe_set_shifts(plan: int, scan: int, d_shifts) -> None:
    """d_shifts: device address (int) of F int32 AP shifts, or None."""
    lib = load()
    _check(lib.fringe_set_shifts(c_void_p(plan), c_int32(int(scan)), c_void_p(d_shifts or None)),
           "fringe_set_shifts")


def fringe_plan_set_chunk(plan: int, scan: int, chunk: int) -> None:
    """APs per work item of scan's search (0: automatic); before the first search."""
    lib = load()
    _check(lib.fringe_plan_set_chunk(c_void_p(plan), c_int32(int(scan)), c_int32(int(chunk))),
           "fringe_plan_set_chunk")


def fringe_plan_get_chunk(plan: int, scan: int) -> int:
    lib = load()
    out = c_int32(0)
    _check(lib.fringe_plan_get_chunk(c_void_p(plan), c_int32(int(scan)), ctypes.byref(out)),
           "fringe_plan_get_chunk")
    return int(out.value)


def fringe_monotonic_ns() -> int:
    """The library's clock (CLOCK_MONOTONIC, ns): time.perf_counter()'s on Linux."""
    return int(load().fringe_monotonic_ns())


def fringe_server_create(subs, window_aps, *, pad_freq=4, pad_time=2, snr_threshold=4.5,
                         max_candidates=1 << 16, flags=0, time_chunk=0, max_inflight=0) -> int:
    """A native continuous-batching server (fringe_serve.h); returns its handle."""
    lib = load()
    sa = _scan_array(subs)
    p, _keep = _params(window_aps, pad_freq, pad_time, snr_threshold, 0, max_candidates, flags)
    out = c_void_p()
    _check(lib.fringe_server_create(sa, len(subs), ctypes.byref(p), int(time_chunk),
                                    int(max_inflight), ctypes.byref(out)), "fringe_server_create")
    return out.value


def fringe_server_set_shifts(server: int, sub: int, d_shifts) -> None:
    _check(load().fringe_server_set_shifts(c_void_p(server), c_int32(int(sub)),
                                           c_void_p(d_shifts or None)), "fringe_server_set_shifts")


def fringe_server_submit(server: int, sub: int, tag: int, d_chunk: int) -> None:
    _check(load().fringe_server_submit(c_void_p(server), c_int32(int(sub)), c_int64(int(tag)),
                                       c_void_p(int(d_chunk) or None)), "fringe_server_submit")


def fringe_server_poll(server: int, res=None, cands=None):
    """Finished chunks: (list of result dicts, candidate records concatenated
    in the same order).  res / cands: reusable buffers (a ctypes array of
    fringe_serve_result, a CANDIDATE_DTYPE array); the candidates returned
    are a view of cands (a new array when it had to grow)."""
    lib = load()
    if res is None:
        res = (fringe_serve_result * 64)()
    if cands is None:
        cands = np.empty(1 << 16, dtype=CANDIDATE_DTYPE)
    n_out, n_c = c_int32(0), c_int64(0)
    rc = lib.fringe_server_poll(c_void_p(server), res, len(res), ctypes.byref(n_out),
                                cands.ctypes.data_as(c_void_p), len(cands), ctypes.byref(n_c))
    if rc == FRINGE_E_CAPACITY:
        return fringe_server_poll(server, res, np.empty(int(n_c.value), dtype=CANDIDATE_DTYPE))
    _check(rc, "fringe_server_poll")
    out = [{k: getattr(res[i], k) for k, _ in fringe_serve_result._fields_}
           for i in range(n_out.value)]
    return out, cands[:n_c.value]


def fringe_server_pending(server: int) -> int:
    n = c_int64(0)
    _check(load().fringe_server_pending(c_void_p(server), ctypes.byref(n)), "fringe_server_pending")
    return int(n.value)


def fringe_server_destroy(server: int) -> None:
    _check(load().fringe_server_destroy(c_void_p(server)), "fringe_server_destroy")


def fringe_search_noalloc(scan: dict, window_aps, d_vis: int, d_out: int, capacity: int,
                          d_total: int, pad_freq=4, pad_time=2, snr_threshold=4.5, flags=0,
                          stream: int = 0) -> None:
    """Enqueue the allocation-free search of one scan: candidates into the
    device array d_out (capacity records), the total into the device int64
    d_total."""
    lib = load()
    sa = _scan_array([scan])
    p, keep = _params(window_aps, pad_freq, pad_time, snr_threshold, 0, 0, flags)
    _check(lib.fringe_search_noalloc(sa, ctypes.byref(p), c_void_p(int(d_vis)),
                                     c_void_p(int(d_out) if d_out else None), int(capacity),
                                     c_void_p(int(d_total)),
                                     c_void_p(int(stream) if stream else None)),
           "fringe_search_noalloc")


def fringe_autospectrum_gains(d_auto: int, n_stations: int, n_spectra: int, n_freq: int,
                              d_pairs: int, n_baselines: int, d_gains_in, d_gains_out: int,
                              stream: int = 0) -> None:
    """Enqueue the auto-spectrum normalisation gains (include/fringe_calib.h):
    d_gains_out[b][f] = g_in[b][f] * (abar_i^2 abar_j^2)^(-1/4); device
    addresses as integers (d_gains_in 0/None: unit gains)."""
    _check(load().fringe_autospectrum_gains(c_void_p(int(d_auto)), int(n_stations),
                                            int(n_spectra), int(n_freq), c_void_p(int(d_pairs)),
                                            int(n_baselines),
                                            c_void_p(int(d_gains_in) if d_gains_in else None),
                                            c_void_p(int(d_gains_out)),
                                            c_void_p(int(stream) if stream else None)),
           "fringe_autospectrum_gains")


def fringe_tune_load(path: str) -> None:
    """Merge a JSON tune table (from fringe_tune_save) into the library's."""
    _check(load().fringe_tune_load(os.fsencode(path)), "fringe_tune_load")


def fringe_tune_save(path: str) -> None:
    """Write the library's tune table as JSON."""
    _check(load().fringe_tune_save(os.fsencode(path)), "fringe_tune_save")


def fringe_tune_clear() -> None:
    load().fringe_tune_clear()


def fringe_plan_tuning(plan: int) -> list:
    """The tune entries (dicts) a FRINGE_AUTOTUNE plan uses."""
    lib = load()
    n = c_int32(0)
    lib.fringe_plan_tuning(c_void_p(plan), None, 0, ctypes.byref(n))
    arr = (fringe_tune_entry * max(1, n.value))()
    _check(lib.fringe_plan_tuning(c_void_p(plan), arr, n.value, ctypes.byref(n)),
           "fringe_plan_tuning")
    return [{k: getattr(arr[i], k) for k, _ in fringe_tune_entry._fields_} for i in range(n.value)]


def fringe_plan_destroy(plan: int) -> None:
    if plan:
        load().fringe_plan_destroy(c_void_p(plan))


def as_candidates(records: np.ndarray) -> np.ndarray:
    """Records with the candidate fields (any field order or widths, extra
    fields ignored) as a contiguous CANDIDATE_DTYPE array, copied by name."""
    if records.dtype == CANDIDATE_DTYPE:
        return np.ascontiguousarray(records)
    out = np.zeros(len(records), CANDIDATE_DTYPE)
    for name in CANDIDATE_DTYPE.names:
        if name in records.dtype.names:
            out[name] = records[name]
        elif name != "reserved":
            raise ValueError(f"candidate records lack the field {name!r}")
    return out


def fringe_match(candidates: np.ndarray, min_windows: int = 2, min_baselines: int = 5):
    """Single pulses from a candidate list (CANDIDATE_DTYPE records):
    (rows as a PULSE_DTYPE array in (pulse, baseline) order, number of pulses)."""
    lib = load()
    c = as_candidates(candidates)
    p = fringe_match_params(int(min_windows), int(min_baselines))
    n_rows, n_pulses = c_int64(0), c_int64(0)
    cptr = c.ctypes.data_as(c_void_p) if len(c) else None
    rc = lib.fringe_match(cptr, len(c), ctypes.byref(p), None, 0, ctypes.byref(n_rows),
                          ctypes.byref(n_pulses))
    if rc not in (FRINGE_OK, FRINGE_E_CAPACITY) or (rc == FRINGE_E_CAPACITY and n_rows.value == 0):
        _check(rc, "fringe_match")
    out = np.zeros(n_rows.value, PULSE_DTYPE)
    if n_rows.value:
        _check(lib.fringe_match(cptr, len(c), ctypes.byref(p), out.ctypes.data_as(c_void_p),
                                len(out), ctypes.byref(n_rows), ctypes.byref(n_pulses)),
               "fringe_match")
    return out, int(n_pulses.value)


def _f64(v) -> np.ndarray:
    return np.ascontiguousarray(v, dtype=np.float64)


def fringe_localize(tau, dtau_dra, dtau_ddec):
    """Eq. (2) least squares: (sol (2,), rms, loo (n, 2), loo_rms (n,));
    the leave-one-out arrays are empty for two baselines."""
    t, a, d = _f64(tau).ravel(), _f64(dtau_dra).ravel(), _f64(dtau_ddec).ravel()
    if not (len(t) == len(a) == len(d)):
        raise ValueError("tau and the partials must have the same length")
    n = len(t)
    sol, rms = np.zeros(2), c_double(0)
    loo, loo_rms = np.zeros((n, 2)), np.zeros(n)
    dp = POINTER(c_double)
    _check(load().fringe_localize(t.ctypes.data_as(dp), a.ctypes.data_as(dp), d.ctypes.data_as(dp),
                                  n, sol.ctypes.data_as(dp), ctypes.byref(rms),
                                  loo.ctypes.data_as(dp), loo_rms.ctypes.data_as(dp)),
           "fringe_localize")
    if n < 3:
        loo, loo_rms = loo[:0], loo_rms[:0]
    return sol, rms.value, loo, loo_rms


def fringe_delay_partials(b_xyz, gast: float, ra: float, dec: float):
    """(dtau/dra, dtau/ddec) in s/rad for Earth-fixed baseline vectors (n, 3) in metres."""
    b = _f64(b_xyz).reshape(-1, 3)
    n = len(b)
    da, dd = np.zeros(n), np.zeros(n)
    dp = POINTER(c_double)
    _check(load().fringe_delay_partials(b.ctypes.data_as(dp), n, float(gast), float(ra),
                                        float(dec), da.ctypes.data_as(dp), dd.ctypes.data_as(dp)),
           "fringe_delay_partials")
    return da, dd


def fringe_dedisperse(d_in: int, d_out: int, n_baselines: int, n_ap: int, n_freq: int,
                      d_shifts: int, stream: int = 0) -> None:
    """Enqueue the dedispersion pass: d_out[b][t][f] = d_in[b][t + d_f][f]."""
    _check(load().fringe_dedisperse(c_void_p(d_in), c_void_p(d_out), int(n_baselines), int(n_ap),
                                    int(n_freq), c_void_p(d_shifts),
                                    c_void_p(int(stream) if stream else None)),
           "fringe_dedisperse")


def fringe_probe_fma(n_blocks: int, iters: int, d_out: int, stream: int = 0) -> float:
    """Enqueue the FP32 FMA-loop probe; returns the flops of the launch."""
    fl = c_double(0)
    _check(load().fringe_probe_fma(int(n_blocks), int(iters), c_void_p(d_out), ctypes.byref(fl),
                                   c_void_p(int(stream) if stream else None)), "fringe_probe_fma")
    return fl.value


def fringe_probe_copy(d_src: int, d_dst: int, nbytes: int, stream: int = 0) -> None:
    """Enqueue the HBM copy probe (nbytes read and nbytes written)."""
    _check(load().fringe_probe_copy(c_void_p(d_src), c_void_p(d_dst), int(nbytes),
                                    c_void_p(int(stream) if stream else None)), "fringe_probe_copy")


class Plan:
    """Owning wrapper of a plan handle (destroyed on close / garbage collection)."""

    def __init__(self, scans: Sequence[dict], window_aps, **kw):
        self.scans = [dict(s) for s in scans]
        self.window_aps = list(window_aps)
        self.kw = dict(kw)
        self.handle = fringe_plan(self.scans, self.window_aps, **kw)

    def search(self, vis_ptrs, stream: int = 0):
        fringe_search(self.handle, vis_ptrs, stream)

    def candidates(self, capacity=None):
        return candidates_get(self.handle, capacity)

    def windows(self, ids):
        return fringe_windows_get(self.handle, ids)

    def window_id(self, scan, baseline, window_ap, t_start):
        return fringe_window_id(self.handle, scan, baseline, window_ap, t_start)

    def grid(self, window_id, m_t, m_f):
        return fringe_grid_get(self.handle, window_id, m_t, m_f)

    def info(self):
        return fringe_plan_info(self.handle)

    def set_gains(self, scan, d_gains):
        fringe_set_gains(self.handle, scan, d_gains)

    def set_shifts(self, scan, d_shifts):
        fringe_set_shifts(self.handle, scan, d_shifts)

    def set_chunk(self, scan, chunk):
        fringe_plan_set_chunk(self.handle, scan, chunk)

    def chunk(self, scan=0):
        return fringe_plan_get_chunk(self.handle, scan)

    def profile(self):
        return fringe_profile_get(self.handle)

    def tuning(self):
        return fringe_plan_tuning(self.handle)

    def close(self):
        if self.handle:
            fringe_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
