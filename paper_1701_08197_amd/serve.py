"""Streaming flagging service with continuous batching.

Stations deliver one request per observation second: that station's subband
blocks (channels x times of complex int8 voltages).  Requests that arrive while
others are on the GPU are admitted as soon as arena slots free up and packed
into the next lof_flag_blocks call; calls alternate between HIP streams so their
work overlaps on the device.  The history flagger's state (per station, subband
and channel) stays on the device inside the lof context, and each call commits
its staged history values in the same enqueue (LOF_OPT_AUTOCOMMIT).  A station's
next second is admitted only after its previous second has completed, so every
history stream sees its blocks in arrival order (Sec. 4.1: the history must be
applied in time order even when seconds are processed on different workers).

Inputs are flagged where they landed in device memory; the arena holds the flag
outputs (and bounds how much work is admitted).  A request's inputs may still be
in flight on the producer's stream when it is submitted: submit() records an
event on the caller's current stream and the flagging stream waits on it.
Back-pressure: a request still waiting for admission `max_wait_s` after its
arrival (e.g. one real-time deadline) is shed and counted instead of queueing
without bound, so latency past saturation stays bounded.  Descriptor tables are
built with vectorised numpy writes into the lof_block layout.  All flagging work
runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import _native as N
from .flagger import Flagger, default_params


# numpy view of struct lof_block (include/lof.h)
BLOCK_DTYPE = np.dtype([("data", "<u8"), ("flags", "<u8"), ("dstride", "<i8"), ("fstride", "<i8"),
                        ("C", "<i4"), ("T", "<i4"), ("dtype", "<i4"), ("sid", "<i4")])
assert BLOCK_DTYPE.itemsize == ctypes.sizeof(N.LofBlock)


@dataclass
class Request:
    station: int
    second: int
    arrival: float                      # host clock (seconds)
    sources: list                       # per subband: device tensor [C, T, 2] int8 (input)
    done: float = 0.0
    slots: list = field(default_factory=list)
    ptrs: np.ndarray = None
    ready: object = None                # event on the producer's stream (inputs written)
    admit_seq: int = -1                 # order of admission (debugging, tests)

    def __post_init__(self):
        self.ptrs = np.fromiter((t.data_ptr() for t in self.sources), dtype=np.uint64, count=len(self.sources))


class Service:
    """Continuous-batching flagger over a fixed device arena of `n_slots` blocks."""

    def __init__(self, n_stations: int, max_subbands: int, n_slots: int, C: int = 64, T: int = 3072,
                 n_hip_streams: int = 2, keep_outputs: bool = False, device: int = 0,
                 max_wait_s: float | None = None, **param_overrides):
        import torch
        self.torch = torch
        self.C, self.T = C, T
        self.max_subbands = max_subbands
        self.dev = torch.device("cuda", device)
        self.out = torch.empty((n_slots, C, T), dtype=torch.uint8, device=self.dev)
        self.out_ptr = np.uint64(self.out.data_ptr()) + np.arange(n_slots, dtype=np.uint64) * np.uint64(C * T)
        self.table = np.zeros(n_slots, dtype=BLOCK_DTYPE)
        self.table["dstride"] = T
        self.table["fstride"] = T
        self.table["C"] = C
        self.table["T"] = T
        self.table["dtype"] = N.LOF_CI8
        self.free = collections.deque(range(n_slots))
        self.n_slots = n_slots
        opts = param_overrides.pop("options", 0) | N.LOF_OPT_AUTOCOMMIT
        prm = default_params(max_streams=n_stations * max_subbands, max_channels=C,
                             max_blocks_per_call=n_slots, max_samples_per_call=n_slots * C * T,
                             options=opts, **param_overrides)
        self.fl = Flagger(prm, device=device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_hip_streams)]
        self.next_stream = 0
        self.queue: collections.deque = collections.deque()
        self.inflight: list = []            # (event, [requests])
        self.busy_station: set = set()
        self.completed: list = []
        self.keep_outputs = keep_outputs
        self.outputs: dict = {}             # (station, second, subband) -> host uint8 array
        self.max_wait_s = max_wait_s
        self.shed = 0                       # requests dropped by back-pressure
        self.n_admitted = 0

    # ---------------------------------------------------------------- admission
    def submit(self, req: Request) -> None:
        if len(req.sources) > self.n_slots:
            raise ValueError(f"request needs {len(req.sources)} blocks, the arena has {self.n_slots}")
        req.ready = self.torch.cuda.Event()
        req.ready.record(self.torch.cuda.current_stream(self.dev))
        self.queue.append(req)

    def _admit(self) -> None:
        batch, need_free = [], 0
        waiting = collections.deque()
        stations_in_batch = set()
        blocked = set()                     # stations with an earlier request still waiting
        now = time.perf_counter()
        while self.queue:
            r = self.queue.popleft()
            n = len(r.sources)
            if self.max_wait_s is not None and now - r.arrival > self.max_wait_s:
                self.shed += 1              # past its deadline before admission
                continue
            if (r.station in self.busy_station or r.station in stations_in_batch or r.station in blocked
                    or need_free + n > len(self.free)):
                waiting.append(r)
                blocked.add(r.station)      # its later seconds must not overtake it
                continue
            batch.append(r)
            r.admit_seq = self.n_admitted
            self.n_admitted += 1
            stations_in_batch.add(r.station)
            need_free += n
        # keep arrival order of everything not admitted
        self.queue = waiting
        if not batch:
            return
        torch = self.torch
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        tab = self.table[:need_free]
        k = 0
        for r in batch:
            n = len(r.sources)
            r.slots = [self.free.popleft() for _ in range(n)]
            tab["data"][k:k + n] = r.ptrs
            tab["flags"][k:k + n] = self.out_ptr[r.slots]
            tab["sid"][k:k + n] = r.station * self.max_subbands + np.arange(n, dtype=np.int32)
            k += n
        for r in batch:
            s.wait_event(r.ready)
            for t in r.sources:
                t.record_stream(s)
        arr = ctypes.cast(tab.ctypes.data, ctypes.POINTER(N.LofBlock))
        rc = self.fl.flag_blocks_raw(arr, need_free, s.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"lof_flag_blocks failed with {rc}")
        ev = torch.cuda.Event()
        ev.record(s)
        for r in batch:
            self.busy_station.add(r.station)
        self.inflight.append((ev, batch))

    def _reap(self) -> int:
        done = 0
        still = []
        now = time.perf_counter()
        for ev, batch in self.inflight:
            if ev.query():
                for r in batch:
                    r.done = now
                    if self.keep_outputs:
                        for sb, slot in enumerate(r.slots):
                            self.outputs[(r.station, r.second, sb)] = self.out[slot].cpu().numpy()
                    self.free.extend(r.slots)
                    self.busy_station.discard(r.station)
                    self.completed.append(r)
                    done += 1
            else:
                still.append((ev, batch))
        self.inflight = still
        return done

    # ---------------------------------------------------------------- driving
    def run(self, arrivals, make_sources, speedup: float = 1.0, poll_s: float = 2e-4):
        """arrivals: sorted (t_obs_seconds, station, second); make_sources(station, second)
        -> list of device tensors.  Observation time runs `speedup` times faster than
        the wall clock.  Returns the completed requests."""
        t0 = time.perf_counter()
        i = 0
        n = len(arrivals)
        while i < n or self.queue or self.inflight:
            now = time.perf_counter()
            while i < n and arrivals[i][0] / speedup <= now - t0:
                t_obs, st, sec = arrivals[i]
                self.submit(Request(st, sec, t0 + t_obs / speedup, make_sources(st, sec)))
                i += 1
            self._reap()
            self._admit()
            if self.inflight or self.queue or i < n:
                nxt = arrivals[i][0] / speedup + t0 if i < n else now + poll_s
                time.sleep(max(0.0, min(poll_s, nxt - time.perf_counter())))
        self.torch.cuda.synchronize()
        return self.completed

    def close(self) -> None:
        self.fl.close()


def latency_summary(completed, C: int, T: int, wall_s: float, deadline_s: float) -> dict:
    lat = sorted(r.done - r.arrival for r in completed)
    if not lat:
        return {}
    def pct(q):
        return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
    samples = sum(len(r.slots) for r in completed) * C * T
    return {"requests": len(lat), "p50_ms": pct(0.5) * 1e3, "p99_ms": pct(0.99) * 1e3,
            "max_ms": lat[-1] * 1e3, "deadline_ms": deadline_s * 1e3,
            "admitted_gsamples_per_s": samples / wall_s / 1e9}
