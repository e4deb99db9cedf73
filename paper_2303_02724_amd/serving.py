"""Continuous-batching request loop for extremum graphs on one GPU.

Requests arrive over time; each names a field that is already on the device
(the "client data").  The loop admits arrived requests while a slot is free
and their HBM footprint fits the budget, groups the admitted ones into a
batch, and launches the batch with ``eg_build_batched`` (a single request
with ``eg_build``) on one of several streams, so batches that start while
others are still running overlap on the device.  Each request keeps its
labels and arc buffers on the device until the caller consumes them.
Latency is measured from a request's arrival to the moment the host sees its
batch complete.

All computation goes through the HIP library; this module only schedules.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field as dc_field

import torch

from . import eg


@dataclass
class Done:
    index: int
    shape: tuple
    arrival: float
    start: float
    end: float
    batch: int
    builder: "eg.Builder"

    @property
    def latency(self):
        return self.end - self.arrival


@dataclass
class ServeStats:
    done: list = dc_field(default_factory=list)
    batches: int = 0
    max_inflight: int = 0
    peak_bytes: int = 0
    rejected_for_memory: int = 0
    regrown: int = 0
    wall_s: float = 0.0

    def summary(self):
        import numpy as np

        lat = np.array([d.latency for d in self.done]) * 1e3
        nvert = sum(int(np_prod(d.shape)) for d in self.done)
        span = max(d.end for d in self.done) - min(d.arrival for d in self.done)
        return {
            "requests": len(self.done),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()),
            "vertices_per_s": nvert / span,
            "batches": self.batches,
            "mean_batch": len(self.done) / max(1, self.batches),
            "max_inflight_batches": self.max_inflight,
            "peak_footprint_gb": self.peak_bytes / 1e9,
            "admission_waits_for_memory": self.rejected_for_memory,
            "capacity_regrowths": self.regrown,
        }


def np_prod(shape):
    p = 1
    for s in shape:
        p *= int(s)
    return p


def footprint(b: "eg.Builder") -> int:
    """Device bytes a request holds while admitted: its field and every
    buffer of its builder."""
    t = 4 * b.n  # the field
    for x in (b.labels, b.ptr, b.maxima, b.saddles, b.beta, b.offsets, b.arcs, b.header, b.ws):
        if x is not None:
            t += x.numel() * x.element_size()
    return t


class _Lane:
    """A stream with its batch workspace and pinned plan buffer."""

    def __init__(self, device):
        self.stream = torch.cuda.Stream(device=device)
        self.batch = None
        self.event = None
        self.bb = None


class Server:
    """Continuous batching over a fixed set of device-resident fields.

    max_slots: requests admitted at once; max_batch: requests per launch;
    lanes: batches in flight at once (one stream each); hbm_budget: bytes of
    admitted footprint.  Builders (per-request buffers) are reused per shape,
    so steady state allocates nothing.
    """

    def __init__(self, device=None, hbm_budget=64 << 30, max_slots=64, max_batch=32, lanes=2, caps_for=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.lanes = [_Lane(self.device) for _ in range(lanes)]
        self.free = {}
        self.caps_for = caps_for or (lambda shape: {})
        self.used = 0
        self.admitted = 0

    def _builder(self, shape):
        lst = self.free.get(shape)
        if lst:
            return lst.pop()
        return eg.Builder(shape, device=self.device, **self.caps_for(shape))

    def _release(self, b):
        self.free.setdefault(b.shape, []).append(b)

    def prewarm(self, shapes, per_shape=1):
        for sh in shapes:
            for _ in range(per_shape):
                self._release(eg.Builder(sh, device=self.device, **self.caps_for(sh)))

    def run(self, requests, fields, on_done=None) -> ServeStats:
        """requests: list of (arrival_s, field_index), sorted by arrival;
        fields: device tensors.  Returns per-request completion records."""
        st = ServeStats()
        pending = list(requests)
        qi = 0
        waiting = []  # admitted, not yet launched: (req index, builder, arrival)
        t0 = time.perf_counter()
        finished = 0
        total = len(pending)
        while finished < total:
            now = time.perf_counter() - t0
            # completions
            for lane in self.lanes:
                if lane.event is not None and lane.event.query():
                    end = time.perf_counter() - t0
                    for (ri, b, arr, start, fi) in lane.batch:
                        h = b.header_values()
                        if h[eg.H_STATUS] == eg.EG_ERR_CAPACITY:
                            # outputs did not fit: grow this request's buffers
                            # and run it again in a later batch
                            self.used -= footprint(b)
                            b.grow(h)
                            self.used += footprint(b)
                            st.peak_bytes = max(st.peak_bytes, self.used)
                            st.regrown += 1
                            waiting.insert(0, (ri, b, arr, fi))
                            continue
                        if h[eg.H_STATUS] != eg.EG_OK:
                            raise eg.EGError(h[eg.H_STATUS], f"request {ri}")
                        st.done.append(Done(ri, b.shape, arr, start, end, st.batches, b))
                        self.used -= footprint(b)
                        self.admitted -= 1
                        finished += 1
                        if on_done is not None:
                            on_done(ri, b)
                        self._release(b)
                    lane.batch = None
                    lane.event = None
            # admission of arrived requests
            while qi < total and pending[qi][0] <= now and self.admitted < self.max_slots:
                arr, fi = pending[qi]
                b = self._builder(tuple(fields[fi].shape))
                need = footprint(b)
                if self.used + need > self.budget and self.admitted > 0:
                    self._release(b)
                    st.rejected_for_memory += 1
                    break
                self.used += need
                self.admitted += 1
                st.peak_bytes = max(st.peak_bytes, self.used)
                waiting.append((qi, b, arr, fi))
                qi += 1
            # launch on a free lane
            lane = next((l for l in self.lanes if l.event is None), None)
            if waiting and lane is not None:
                batch, waiting = waiting[: self.max_batch], waiting[self.max_batch:]
                start = time.perf_counter() - t0
                s = lane.stream
                if len(batch) == 1:
                    ri, b, arr, fi = batch[0]
                    b.launch(fields[fi], stream=s)
                else:
                    bb = eg.BatchBuilder.from_builders([b for (_, b, _, _) in batch], device=self.device,
                                                       reuse=lane.bb)
                    bb.plan([fields[fi] for (_, _, _, fi) in batch], stream=s)
                    bb.launch(stream=s)
                    lane.bb = bb
                ev = torch.cuda.Event()
                ev.record(s)
                lane.event = ev
                lane.batch = [(ri, b, arr, start, fi) for (ri, b, arr, fi) in batch]
                st.batches += 1
                st.max_inflight = max(st.max_inflight, sum(l.event is not None for l in self.lanes))
                continue
            if not waiting and all(l.event is None for l in self.lanes) and qi < total:
                # idle until the next arrival
                dt = pending[qi][0] - (time.perf_counter() - t0)
                if dt > 2e-4:
                    time.sleep(dt - 1e-4)
        st.wall_s = time.perf_counter() - t0
        return st
