"""Continuous-batching server for reference-bank correlation requests.

A request is one received pulse (n complex samples) and its scale count J;
its result is the planes of every eligible bank reference (E x J x N).
The bank (plans and split MFMA weights) stays resident on the device.

Serving loop (host side; all arithmetic runs in libsidwt's kernels):
  * arrivals are released into a FIFO queue at their arrival time;
  * admission: while a slot (a HIP stream with its own bank workspace) is
    free, the queue head is admitted if the bytes of everything in flight
    plus its own footprint (pulse + planes + scratch pyramid) stay within
    the HBM budget; all requests admitted at that moment form one group
    (continuous batching) and go to the GPU as one bank call on the free
    slot, after an asynchronous copy of their pulses from pinned memory;
  * a request larger than the whole budget is admitted alone once nothing
    else is in flight, so nothing is ever dropped;
  * each slot keeps a device arena for its group's pulses and one for its
    planes (grown only when a larger group arrives, so a steady serving
    loop makes no device allocations); a group's tensors are views into
    them, reused once the group has completed;
  * slots overlap on the device; completion is detected by polling an
    event per group, which frees the group's bytes and its slot;
  * latency = completion (event timestamp on the device clock, anchored to
    the host clock at start) - arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float             # seconds after the start of the run
    rx: object                 # pinned host complex64 torch tensor (n,)
    J: int
    keep: bool = False         # keep the device output for inspection


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    arrival: float
    admitted: float
    completed: float
    group: int
    slot: int

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class Server:
    def __init__(self, bank, slots: int = 4, budget_bytes: int = 8 << 30,
                 max_group: int = 64, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.bank = bank
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.ws = [bank.workspace() for _ in range(slots)]
        self.budget = int(budget_bytes)
        self.max_group = max_group
        self.outputs = {}
        self.max_inflight_bytes = 0
        self.in_arena = [None] * slots
        self.out_arena = [None] * slots
        self.arena_grows = 0

    def _arena_bytes(self) -> int:
        return sum(b.numel() * 8 for arenas in (self.in_arena, self.out_arena)
                   for b in arenas if b is not None)

    def _arena(self, arenas, slot: int, nelem: int, busy):
        """The slot's arena with room for nelem complex64 values (called only
        while the slot is idle, so the old buffer is no longer in use).  When
        the arenas together would pass the HBM budget, those of idle slots
        are released first."""
        buf = arenas[slot]
        if buf is None or buf.numel() < nelem:
            old = 0 if buf is None else buf.numel()
            arenas[slot] = None
            want = max(nelem, old + old // 4)
            if self._arena_bytes() + 8 * want > self.budget:
                for a in (self.in_arena, self.out_arena):
                    for s in range(len(a)):
                        if s != slot and s not in busy:
                            a[s] = None
                if self._arena_bytes() + 8 * want > self.budget:
                    want = nelem
            arenas[slot] = self.torch.empty(want, dtype=self.torch.complex64, device=self.device)
            self.arena_grows += 1
        return arenas[slot]

    def _views(self, slot: int, group, busy):
        """Device tensors of one group: its pulses (copied from pinned host
        memory on the slot's stream) and its planes, carved from the slot's
        arenas."""
        from . import transform_length
        ns = [r.rx.numel() for r in group]
        shapes = []
        for r, n in zip(group, ns):
            shapes.append((self.bank.eligible(n), r.J, transform_length(n, r.J)))
        # planes start on even elements (16-byte aligned)
        sizes = [e * j * N for e, j, N in shapes]
        sizes = [s + (s & 1) for s in sizes]
        ain = self._arena(self.in_arena, slot, sum(ns), busy)
        aout = self._arena(self.out_arena, slot, max(1, sum(sizes)), busy)
        rx, outs, oi, oo = [], [], 0, 0
        for r, n, shp, sz in zip(group, ns, shapes, sizes):
            x = ain[oi:oi + n]
            x.copy_(r.rx, non_blocking=True)
            rx.append(x)
            outs.append(aout[oo:oo + shp[0] * shp[1] * shp[2]].view(shp))
            oi += n
            oo += sz
        return rx, outs

    def footprint(self, n: int, J: int) -> int:
        from . import transform_length
        E = self.bank.eligible(n)
        return n * 8 + E * J * transform_length(n, J) * 8 + self.bank.scratch_bytes(n, J)

    def run(self, requests, idle_sleep: float = 20e-6):
        """Serve `requests` (any order; sorted by arrival here).  Returns a
        list of Record, one per request, in completion order.  Python's
        cyclic garbage collector is paused for the run (a full collection
        over the run's objects stalls the loop for tens of milliseconds)."""
        import gc
        enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, idle_sleep)
        finally:
            if enabled:
                gc.enable()

    def _run(self, requests, idle_sleep):
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        fp = {r.rid: self.footprint(r.rx.numel(), r.J) for r in reqs}
        start = torch.cuda.Event(enable_timing=True)
        start.record(self.streams[0])
        start.synchronize()
        t0 = time.perf_counter()
        pending = collections.deque()
        inflight = {}            # slot -> (event, group, bytes, admitted_time, gid, outs)
        used = 0
        nxt = 0
        gid = 0
        records = []
        while len(records) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            progressed = False
            for slot in list(inflight):
                ev, group, nbytes, adm, g, outs = inflight[slot]
                if ev.query():
                    done = start.elapsed_time(ev) * 1e-3
                    for r, o in zip(group, outs):
                        records.append(Record(r.rid, r.rx.numel(), r.arrival, adm, done, g, slot))
                        if r.keep:
                            self.outputs[r.rid] = o
                    used -= nbytes
                    del inflight[slot]
                    progressed = True
            free = [s for s in range(len(self.streams)) if s not in inflight]
            if free and pending:
                group, nbytes = [], 0
                while pending and len(group) < self.max_group:
                    b = fp[pending[0].rid]
                    if used + nbytes + b <= self.budget or (not inflight and not group):
                        group.append(pending.popleft())
                        nbytes += b
                    else:
                        break
                if group:
                    slot = free[0]
                    st = self.streams[slot]
                    adm = time.perf_counter() - t0
                    with torch.cuda.stream(st):
                        rx, outs = self._views(slot, group, inflight)
                        self.bank.correlate(rx, [r.J for r in group], out=outs, stream=st,
                                            workspace=self.ws[slot])
                        # kept results leave the arena before the slot is reused
                        outs = [o.clone() if r.keep else None for r, o in zip(group, outs)]
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(st)
                    inflight[slot] = (ev, group, nbytes, adm, gid, outs)
                    gid += 1
                    used += nbytes
                    self.max_inflight_bytes = max(self.max_inflight_bytes, used)
                    progressed = True
            if not progressed:
                if nxt < len(reqs) and not pending and not inflight:
                    # idle until the next arrival
                    wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(idle_sleep)
        return records

    def close(self):
        self.torch.cuda.synchronize()
        for w in self.ws:
            w.free()
        self.ws = []
        self.in_arena = [None] * len(self.streams)
        self.out_arena = [None] * len(self.streams)


def summarize(records, t_end=None) -> dict:
    lat = np.array([r.latency for r in records])
    samples = sum(r.n for r in records)
    t_first = min(r.arrival for r in records)
    t_last = max(r.completed for r in records) if t_end is None else t_end
    span = max(t_last - t_first, 1e-9)
    return {"requests": len(records), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "samples_per_s": samples / span, "requests_per_s": len(records) / span,
            "groups": len({r.group for r in records})}
