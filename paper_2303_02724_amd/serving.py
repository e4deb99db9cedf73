"""Continuous-batching request loop for extremum graphs on one GPU.

Requests arrive over time; each names a field, normally in pinned host memory
(the client's data).  The loop admits arrived requests while a slot is free
and their device footprint fits the budget; at admission the field is copied
to the request's device buffer on a copy stream.  Requests whose copies have
landed are grouped into a batch and launched with ``eg_build_batched`` (a
single request with ``eg_build``) on one of several compute streams, so
batches that start while others are still running overlap on the device,
and so does the copy of the next request with the compute of earlier ones.
Each request keeps its labels and arc buffers on the device until the caller
consumes them.  Latency is measured from a request's arrival to the moment
the host sees its batch complete, so it includes the copy.

Memory: ``used`` is every byte the server holds on the device, the buffers
of admitted requests and the pooled buffers kept for reuse alike.  A request
reuses a pooled buffer set of its shape when one is free; otherwise its
footprint is computed from the shape before anything is allocated, pooled
sets of other shapes are released until it fits, and if it still does not
fit the request waits (unless nothing is admitted, when it is let through).

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
    batch: int  # launch number of its batch
    size: int   # requests in that batch
    builder: "eg.Builder"

    @property
    def latency(self):
        return self.end - self.arrival


@dataclass
class ServeStats:
    done: list = dc_field(default_factory=list)
    batches: int = 0
    batch_sizes: list = dc_field(default_factory=list)
    max_inflight: int = 0
    peak_bytes: int = 0
    admission_waits_for_memory: int = 0
    pool_evictions: int = 0
    regrown: int = 0
    copied_bytes: int = 0
    wall_s: float = 0.0

    def summary(self):
        import numpy as np

        lat = np.array([d.latency for d in self.done]) * 1e3
        nvert = sum(int(np_prod(d.shape)) for d in self.done)
        span = max(d.end for d in self.done) - min(d.arrival for d in self.done)
        sizes = np.array(self.batch_sizes) if self.batch_sizes else np.zeros(1)
        return {
            "requests": len(self.done),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()),
            "vertices_per_s": nvert / span,
            "batches": self.batches,
            "mean_batch": len(self.done) / max(1, self.batches),
            "max_batch": int(sizes.max()),
            "batches_of_more_than_one": int((sizes > 1).sum()),
            "max_inflight_batches": self.max_inflight,
            "peak_footprint_gb": self.peak_bytes / 1e9,
            "admission_waits_for_memory": self.admission_waits_for_memory,
            "pool_evictions": self.pool_evictions,
            "capacity_regrowths": self.regrown,
            "h2d_gb": self.copied_bytes / 1e9,
        }


def np_prod(shape):
    p = 1
    for s in shape:
        p *= int(s)
    return p


def footprint(b: "eg.Builder") -> int:
    """Device bytes of one request's buffer set: its field copy and every
    buffer of its builder."""
    t = 0
    for x in (getattr(b, "field_dev", None), b.labels, b.ptr, b.maxima, b.saddles, b.beta, b.offsets, b.arcs,
              b.header, b.ws):
        if x is not None:
            t += x.numel() * x.element_size()
    return t


def footprint_of(shape, caps: dict, want_ptr: bool = False) -> int:
    """The same sum for a buffer set that does not exist yet (host-only)."""
    n = np_prod(shape)
    c = eg.default_caps(n, len(shape))
    c.update({k: int(v) for k, v in caps.items() if v is not None})
    ws = eg.workspace_bytes(shape, c["cap_sad"]) + 256
    i32 = 4 * (n + (n if want_ptr else 0) + max(1, c["cap_max"]) + 2 * max(1, c["cap_sad"]) + c["cap_sad"] + 1 +
               max(1, c["cap_arc"]) + eg.H_SLOTS)
    return 4 * n + i32 + ws


class _Lane:
    """A compute stream with its batch workspace and pinned plan buffer."""

    def __init__(self, device):
        self.stream = torch.cuda.Stream(device=device)
        self.batch = None
        self.event = None
        self.bb = None


@dataclass
class _Req:
    index: int
    builder: "eg.Builder"
    arrival: float
    field: torch.Tensor  # the device field the build reads
    copied: "torch.cuda.Event | None"


class Server:
    """Continuous batching on one GPU.

    max_slots: requests admitted at once; max_batch: requests per launch;
    lanes: batches in flight at once (one stream each); hbm_budget: device
    bytes the server may hold.  Buffer sets (field copy, outputs, workspace)
    are pooled per shape, so steady state allocates nothing.
    """

    def __init__(self, device=None, hbm_budget=64 << 30, max_slots=64, max_batch=32, lanes=2, caps_for=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.lanes = [_Lane(self.device) for _ in range(lanes)]
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.free = {}
        self.caps_for = caps_for or (lambda shape: {})
        self.used = 0  # every device byte held: admitted and pooled buffer sets
        self.admitted = 0

    def _new(self, shape):
        b = eg.Builder(shape, device=self.device, **self.caps_for(shape))
        b.field_dev = torch.empty(shape, dtype=torch.float32, device=self.device)
        self.used += footprint(b)
        return b

    def _release(self, b):
        self.free.setdefault(b.shape, []).append(b)

    def _evict_for(self, need, keep_shape, st):
        """Release pooled buffer sets of other shapes until `need` more bytes
        fit the budget (or none is left)."""
        for shape in list(self.free):
            if shape == keep_shape:
                continue
            lst = self.free[shape]
            while lst and self.used + need > self.budget:
                b = lst.pop()
                self.used -= footprint(b)
                st.pool_evictions += 1
            if not lst:
                del self.free[shape]
            if self.used + need <= self.budget:
                return

    def _acquire(self, shape, st):
        """A buffer set for `shape`: pooled, or new if it fits the budget
        (checked before allocating); None when the request must wait."""
        lst = self.free.get(shape)
        if lst:
            return lst.pop()
        need = footprint_of(shape, self.caps_for(shape))
        if self.used + need > self.budget:
            self._evict_for(need, shape, st)
        if self.used + need > self.budget and self.admitted > 0:
            return None
        return self._new(shape)

    def prewarm(self, shapes, per_shape=1):
        for sh in shapes:
            for _ in range(per_shape):
                self._release(self._new(tuple(sh)))

    def run(self, requests, fields, on_done=None) -> ServeStats:
        """requests: list of (arrival_s, field_index), sorted by arrival;
        fields: host tensors (pinned, copied at admission) or device tensors
        (read in place).  Returns per-request completion records."""
        st = ServeStats()
        pending = list(requests)
        qi = 0
        waiting = []  # admitted, not yet launched
        t0 = time.perf_counter()
        finished = 0
        total = len(pending)
        st.peak_bytes = self.used
        while finished < total:
            now = time.perf_counter() - t0
            # completions
            for lane in self.lanes:
                if lane.event is not None and lane.event.query():
                    end = time.perf_counter() - t0
                    for (r, start, bid, size) in lane.batch:
                        b = r.builder
                        h = b.header_values()
                        if h[eg.H_STATUS] == eg.EG_ERR_CAPACITY:
                            # outputs did not fit: grow this request's buffers
                            # and run it again in a later batch
                            self.used -= footprint(b)
                            b.grow(h)
                            self.used += footprint(b)
                            st.peak_bytes = max(st.peak_bytes, self.used)
                            st.regrown += 1
                            waiting.insert(0, r)
                            continue
                        if h[eg.H_STATUS] != eg.EG_OK:
                            raise eg.EGError(h[eg.H_STATUS], f"request {r.index}")
                        st.done.append(Done(r.index, b.shape, r.arrival, start, end, bid, size, b))
                        self.admitted -= 1
                        finished += 1
                        if on_done is not None:
                            on_done(r.index, b)
                        self._release(b)
                    lane.batch = None
                    lane.event = None
            # admission of arrived requests: buffers, then the copy of the field
            while qi < total and pending[qi][0] <= now and self.admitted < self.max_slots:
                arr, fi = pending[qi]
                src = fields[fi]
                b = self._acquire(tuple(src.shape), st)
                if b is None:
                    st.admission_waits_for_memory += 1
                    break
                self.admitted += 1
                st.peak_bytes = max(st.peak_bytes, self.used)
                if src.is_cuda:
                    waiting.append(_Req(qi, b, arr, src, None))
                else:
                    with torch.cuda.stream(self.copy_stream):
                        b.field_dev.copy_(src, non_blocking=True)
                        ev = torch.cuda.Event()
                        ev.record(self.copy_stream)
                    st.copied_bytes += src.numel() * src.element_size()
                    waiting.append(_Req(qi, b, arr, b.field_dev, ev))
                qi += 1
            # launch the requests whose fields have landed on a free lane
            lane = next((l for l in self.lanes if l.event is None), None)
            if waiting and lane is not None:
                batch, rest = [], []
                for r in waiting:
                    if len(batch) < self.max_batch and (r.copied is None or r.copied.query()):
                        batch.append(r)
                    else:
                        rest.append(r)
                if batch:
                    waiting = rest
                    start = time.perf_counter() - t0
                    s = lane.stream
                    if len(batch) == 1:
                        batch[0].builder.launch(batch[0].field, stream=s)
                    else:
                        bb = eg.BatchBuilder.from_builders([r.builder for r in batch], device=self.device,
                                                           reuse=lane.bb)
                        bb.plan([r.field for r in batch], stream=s)
                        bb.launch(stream=s)
                        lane.bb = bb
                    ev = torch.cuda.Event()
                    ev.record(s)
                    lane.event = ev
                    lane.batch = [(r, start, st.batches, len(batch)) for r in batch]
                    st.batches += 1
                    st.batch_sizes.append(len(batch))
                    st.max_inflight = max(st.max_inflight, sum(l.event is not None for l in self.lanes))
                    continue
            if not waiting and all(l.event is None for l in self.lanes) and qi < total:
                # idle until the next arrival
                dt = pending[qi][0] - (time.perf_counter() - t0)
                if dt > 2e-4:
                    time.sleep(dt - 1e-4)
        st.wall_s = time.perf_counter() - t0
        return st
