"""Continuous-batching fringe search over streamed correlator chunks.

Each subarray is a stream of fixed-length chunks (all baselines x chunk APs x
channels, complex64).  The server keeps, per subarray, a streaming plan of
libfringe (its device-resident history of the last APs, so windows that span
chunk boundaries are searched exactly once) and a HIP stream of default
priority.  Requests are admitted in arrival order as soon as

  * a device input slot is free (slots are what the HBM budget leaves after
    the plans' own memory, one chunk each; a chunk already in HBM is searched
    in place and its slot only bounds how many are in flight), and
  * the subarray's plan is idle (chunks of one subarray are searched in order),

so chunks of different subarrays that arrive while others are on the GPU run
concurrently on their own streams.  A request's latency is the time from its
arrival to its candidate list being on the host.  All search work runs in
libfringe's kernels; this module only moves data into slots, launches and
polls.

FringeBatchServer is the other arrangement: one streaming plan whose scans
are the subarrays, and one search call per step over the next chunk of every
subarray that has one waiting, so one fused launch covers them all (small
subarrays no longer leave the GPU half empty); a chunk that arrives during a
step joins the next one.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from .binding import (CANDIDATE_DTYPE, FRINGE_STREAMING, Plan, fringe_serve_result,
                      fringe_server_create, fringe_server_destroy, fringe_server_pending,
                      fringe_server_poll, fringe_server_set_shifts, fringe_server_submit)


@dataclass
class Request:
    sub: int                 # subarray index
    seq: int                 # chunk number within the subarray
    arrival: float           # seconds on the server clock
    payload: object          # torch tensor [nb][chunk][n_if][n_chan] complex64 (device or pinned host)


@dataclass
class Result:
    sub: int
    seq: int
    arrival: float
    done: float
    candidates: np.ndarray
    n_windows: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    results: List[Result] = field(default_factory=list)
    wall: float = 0.0
    max_inflight: int = 0

    def latencies_ms(self):
        return np.array([r.latency * 1e3 for r in self.results])

    def summary(self) -> dict:
        lat = self.latencies_ms()
        n_win = sum(r.n_windows for r in self.results)
        return {
            "chunks": len(self.results),
            "wall_s": self.wall,
            "chunks_per_s": len(self.results) / self.wall if self.wall > 0 else 0.0,
            "windows_per_s": n_win / self.wall if self.wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "max_inflight": self.max_inflight,
        }


class FringeServer:
    """Continuous-batching server over streaming fringe-search plans."""

    def __init__(self, subarrays: Sequence[dict], window_aps, *, pad_freq: int = 4,
                 pad_time: int = 2, snr_threshold: float = 4.5, hbm_budget_bytes: int = 0,
                 max_candidates: int = 1 << 16, max_slots: Optional[int] = None,
                 time_chunk: int = 0, shifts: Optional[Sequence[object]] = None,
                 device: str = "cuda:0"):
        """time_chunk: APs per work item of every plan's search (0: each
        plan's automatic choice, which sizes it to fill the device alone;
        the plans here share the device, so longer chunks transform fewer
        halo APs).  shifts: per subarray, a device int32 tensor of F
        dedispersion shifts (or None): its chunks are searched dedispersed,
        each call reporting the windows that end max(shift) APs before the
        chunk's end."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.subs = [dict(s) for s in subarrays]
        self.plans = [Plan([s], window_aps, pad_freq=pad_freq, pad_time=pad_time,
                           snr_threshold=snr_threshold, max_candidates=max_candidates,
                           flags=FRINGE_STREAMING) for s in self.subs]
        self.shifts = list(shifts) if shifts is not None else [None] * len(self.subs)
        for p, sh in zip(self.plans, self.shifts):
            if sh is not None:
                p.set_shifts(0, sh.data_ptr())
            if time_chunk:
                p.set_chunk(0, time_chunk)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in self.subs]
        self.chunk_elems = [s["n_baselines"] * s["n_ap"] * s["n_if"] * s["n_chan"] for s in self.subs]
        slot_elems = max(self.chunk_elems)
        plan_bytes = sum(p.info()["device_bytes"] for p in self.plans)
        n_slots = max_slots if max_slots is not None else 2 * len(self.subs)
        if hbm_budget_bytes:
            fit = (int(hbm_budget_bytes) - plan_bytes) // (slot_elems * 8)
            if fit < 1:
                raise MemoryError(f"HBM budget {hbm_budget_bytes} leaves no room for a "
                                  f"{slot_elems * 8}-byte chunk after {plan_bytes} bytes of plans")
            n_slots = min(n_slots, int(fit))
        self.slots = [torch.empty(slot_elems, dtype=torch.complex64, device=self.device)
                      for _ in range(n_slots)]
        self.free = list(range(n_slots))
        # per subarray, its chunks waiting in arrival order
        self.queues = [collections.deque() for _ in self.subs]
        self.busy: Dict[int, tuple] = {}   # sub -> (request, slot, event)
        self.clock0 = time.perf_counter()

    # ---------------------------------------------------------------- api --
    def now(self) -> float:
        return time.perf_counter() - self.clock0

    def submit(self, req: Request) -> None:
        self.queues[req.sub].append(req)

    def inflight(self) -> int:
        return len(self.busy)

    def poll(self) -> List[Result]:
        """Collect finished chunks, then admit waiting ones."""
        out = []
        for sub in list(self.busy):
            req, slot, ev = self.busy[sub]
            if ev.query():
                plan = self.plans[sub]
                cands = plan.candidates()
                n_win = plan.info()["n_windows"]
                out.append(Result(sub, req.seq, req.arrival, self.now(), cands, n_win))
                self.free.append(slot)
                del self.busy[sub]
        self._admit()
        return out

    def close(self):
        for p in self.plans:
            p.close()

    # ---------------------------------------------------------- internals --
    def _admit(self):
        # idle subarrays with a chunk waiting, oldest head first: the
        # first-come order across subarrays, each subarray's chunks in turn
        if not self.free:
            return
        ready = [q[0] for sub, q in enumerate(self.queues) if q and sub not in self.busy]
        ready.sort(key=lambda r: (r.arrival, r.sub))
        for req in ready:
            if not self.free:
                break
            self.queues[req.sub].popleft()
            self._launch(req, self.free.pop())

    def _launch(self, req: Request, slot: int):
        torch = self.torch
        st = self.streams[req.sub]
        n = self.chunk_elems[req.sub]
        pay = req.payload
        if pay.device == self.device and pay.is_contiguous():
            # already in HBM: the plan reads it where it is (the server
            # holds the request until the chunk is done); the slot only
            # counts against the admission budget
            src = pay
            if torch.cuda.current_stream() != st:
                st.wait_stream(torch.cuda.current_stream())
        else:
            src = self.slots[slot][:n].view(pay.shape)
            with torch.cuda.stream(st):
                src.copy_(pay, non_blocking=True)
        self.plans[req.sub].search([src.data_ptr()], st.cuda_stream)
        ev = torch.cuda.Event()
        ev.record(st)
        self.busy[req.sub] = (req, slot, ev)


class FringeNativeServer:
    """The library's native server (fringe_server_*): the same per-subarray
    plans and streams as FringeServer, admitted, launched and collected by
    a worker thread in the library instead of this process's Python loop.
    Chunks must already be in HBM (device tensors); a result's done time is
    when the worker saw its search finish and copied its candidates (the
    library's clock is CLOCK_MONOTONIC, which time.perf_counter reads)."""

    def __init__(self, subarrays: Sequence[dict], window_aps, *, pad_freq: int = 4,
                 pad_time: int = 2, snr_threshold: float = 4.5, max_candidates: int = 1 << 16,
                 time_chunk: int = 0, max_inflight: int = 0,
                 shifts: Optional[Sequence[object]] = None, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.subs = [dict(s) for s in subarrays]
        self.handle = fringe_server_create(self.subs, window_aps, pad_freq=pad_freq,
                                           pad_time=pad_time, snr_threshold=snr_threshold,
                                           max_candidates=max_candidates,
                                           time_chunk=time_chunk, max_inflight=max_inflight)
        self.shifts = list(shifts) if shifts is not None else [None] * len(self.subs)
        for i, sh in enumerate(self.shifts):
            if sh is not None:
                fringe_server_set_shifts(self.handle, i, sh.data_ptr())
        self.held: Dict[int, Request] = {}   # tag -> request (its payload stays alive)
        self.next_tag = 0
        self._res = (fringe_serve_result * 64)()
        self._cands = np.empty(max(1, max_candidates) * 4, dtype=CANDIDATE_DTYPE)
        self.clock0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.clock0

    def submit(self, req: Request) -> None:
        pay = req.payload
        if pay.device != self.device or not pay.is_contiguous():
            raise ValueError("FringeNativeServer takes contiguous chunks already in device memory")
        tag = self.next_tag
        self.next_tag += 1
        self.held[tag] = req
        fringe_server_submit(self.handle, req.sub, tag, pay.data_ptr())

    def inflight(self) -> int:
        return fringe_server_pending(self.handle)

    def poll(self) -> List[Result]:
        res, cands = fringe_server_poll(self.handle, self._res, self._cands)
        if len(cands) and not np.shares_memory(cands, self._cands):
            self._cands = cands.base   # the buffer grew for a large result: keep it
        out, k = [], 0
        for r in res:
            req = self.held.pop(r["tag"])
            if r["status"] != 0:
                raise RuntimeError(f"chunk {req.sub}/{req.seq}: search failed ({r['status']})")
            n = r["n_candidates"]
            out.append(Result(req.sub, req.seq, req.arrival, r["t_done_ns"] * 1e-9 - self.clock0,
                              cands[k:k + n].copy(), r["n_windows"]))
            k += n
        return out

    def close(self):
        if self.handle:
            fringe_server_destroy(self.handle)
            self.handle = None


def run_schedule(server: FringeServer, schedule, payloads, idle_sleep: float = 20e-6) -> ServeStats:
    """Play arrivals (t_seconds, sub, seq) in real time against the server.
    payloads[sub][seq] is the chunk tensor.  Returns per-chunk results."""
    sched = sorted(schedule)
    stats = ServeStats()
    i = 0
    n = len(sched)
    server.clock0 = time.perf_counter()
    while len(stats.results) < n:
        now = server.now()
        while i < n and sched[i][0] <= now:
            t, sub, seq = sched[i]
            server.submit(Request(sub, seq, t, payloads[sub][seq]))
            i += 1
        got = server.poll()
        stats.results.extend(got)
        stats.max_inflight = max(stats.max_inflight, server.inflight())
        if not got and (i >= n or sched[i][0] > server.now()):
            time.sleep(idle_sleep)
    stats.wall = server.now() - (sched[0][0] if sched else 0.0)
    return stats


def poisson_schedule(n_subs: int, n_chunks: int, rate_per_sub: float, seed: int = 0):
    """Arrival times (Poisson per subarray, rate in chunks/s) of n_chunks
    chunks per subarray, in order within each subarray."""
    rng = np.random.default_rng(seed)
    sched = []
    for s in range(n_subs):
        t = np.cumsum(rng.exponential(1.0 / rate_per_sub, n_chunks))
        sched += [(float(t[k]), s, k) for k in range(n_chunks)]
    return sched


def stream_windows(desc: dict, window_aps, seq: int) -> int:
    """Windows a streaming search reports for chunk seq of a subarray: those
    whose last AP lies in the chunk (chunks of desc["n_ap"] APs)."""
    c = int(desc["n_ap"])
    lo, hi = seq * c, (seq + 1) * c          # last AP in [lo, hi)
    n = 0
    for w in window_aps:
        st = max(1, w // 2)
        first = max(0, lo - w + 1)           # start range [first, hi - w]
        last = hi - w
        if last < first:
            continue
        j0 = -(-first // st)
        j1 = last // st
        n += max(0, j1 - j0 + 1)
    return n * int(desc["n_baselines"])


class FringeBatchServer:
    """Continuous-batching server with one launch per step over every
    subarray that has a chunk waiting (the same API as FringeServer)."""

    def __init__(self, subarrays: Sequence[dict], window_aps, *, pad_freq: int = 4,
                 pad_time: int = 2, snr_threshold: float = 4.5, max_candidates: int = 1 << 18,
                 time_chunk: int = 0, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.subs = [dict(s) for s in subarrays]
        self.window_aps = list(window_aps)
        self.plan = Plan(self.subs, window_aps, pad_freq=pad_freq, pad_time=pad_time,
                         snr_threshold=snr_threshold, max_candidates=max_candidates,
                         flags=FRINGE_STREAMING)
        if time_chunk:
            for s in range(len(self.subs)):
                self.plan.set_chunk(s, time_chunk)
        self.stream = torch.cuda.Stream(device=self.device)
        self.slots = [torch.empty(s["n_baselines"] * s["n_ap"] * s["n_if"] * s["n_chan"],
                                  dtype=torch.complex64, device=self.device) for s in self.subs]
        self.queues = [collections.deque() for _ in self.subs]
        self.batch: Optional[tuple] = None    # (requests, event, payload refs)
        self.clock0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.clock0

    def submit(self, req: Request) -> None:
        self.queues[req.sub].append(req)

    def inflight(self) -> int:
        return len(self.batch[0]) if self.batch else 0

    def poll(self) -> List[Result]:
        out = []
        if self.batch is not None and self.batch[1].query():
            reqs = self.batch[0]
            cands = self.plan.candidates()
            done = self.now()
            for r in reqs:
                mine = cands[cands["scan"] == r.sub]
                out.append(Result(r.sub, r.seq, r.arrival, done, mine,
                                  stream_windows(self.subs[r.sub], self.window_aps, r.seq)))
            self.batch = None
        if self.batch is None:
            self._launch()
        return out

    def close(self):
        self.plan.close()

    def _launch(self):
        torch = self.torch
        reqs = [q.popleft() for q in self.queues if q]
        if not reqs:
            return
        st = self.stream
        st.wait_stream(torch.cuda.current_stream())
        ptrs: List[Optional[int]] = [None] * len(self.subs)
        keep = []
        for r in reqs:
            pay = r.payload
            if pay.device == self.device and pay.is_contiguous():
                src = pay
            else:
                src = self.slots[r.sub][:pay.numel()].view(pay.shape)
                with torch.cuda.stream(st):
                    src.copy_(pay, non_blocking=True)
            keep.append(src)
            ptrs[r.sub] = src.data_ptr()
        self.plan.search(ptrs, st.cuda_stream)
        ev = torch.cuda.Event()
        ev.record(st)
        self.batch = (reqs, ev, keep)
