"""Thin Python binding of ``libeg_hip.so`` (the C ABI in ``include/eg.h``).

Argument marshalling only: PyTorch provides device memory and the stream;
every step of the computation runs in the library's HIP kernels.  There is
no CPU path: if the library is missing or no HIP device is present, the
calls raise.

    res = eg.build(field)                # field: CUDA tensor, n = 1..6 axes
                                         # (float32; other types via eg_order_field)
    res.maxima, res.saddles, res.arc_offsets, res.arc_maxima, res.labels

``Builder`` keeps the buffers of one shape allocated so that repeated calls
(benchmarks, serving) allocate nothing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field as dc_field

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeg_hip.so")

(EG_OK, EG_ERR_ARG, EG_ERR_TOO_LARGE, EG_ERR_WORKSPACE, EG_ERR_NAN, EG_ERR_CAPACITY, EG_ERR_HIP, EG_ERR_SCRATCH,
 EG_ERR_UNRESOLVED) = range(9)


def tuning(tile3: int = 0, tile2: int = 0, hops: int = 0, exits_log2: int = 0) -> int:
    """eg_out.tuning value (EG_TUNE_TILE3 | EG_TUNE_TILE2 | EG_TUNE_HOPS |
    EG_TUNE_EXITS)."""
    return (tile3 & 0xF) | ((tile2 & 0xF) << 4) | ((hops & 0xFF) << 8) | ((exits_log2 & 0x1F) << 16)
EG_MINIMA = 0x1
EG_MAX_NDIM = 6
H_STATUS, H_NMAX, H_NSAD, H_NARC, H_NPAIRS, H_PASSES, H_EXITS = range(7)
H_SLOTS = 8


class EGError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"eg status {status} ({status_string(status)}) {msg}".strip())


class eg_out(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("labels", ctypes.c_void_p),
        ("ptr", ctypes.c_void_p),
        ("maxima", ctypes.c_void_p),
        ("cap_max", ctypes.c_int64),
        ("saddles", ctypes.c_void_p),
        ("saddle_beta", ctypes.c_void_p),
        ("arc_offsets", ctypes.c_void_p),
        ("cap_sad", ctypes.c_int64),
        ("arc_maxima", ctypes.c_void_p),
        ("cap_arc", ctypes.c_int64),
        ("workspace", ctypes.c_void_p),
        ("ws_bytes", ctypes.c_size_t),
        ("header", ctypes.c_void_p),
        ("tuning", ctypes.c_uint32),
    ]


class eg_paths_out(ctypes.Structure):
    _fields_ = [
        ("pair_offsets", ctypes.c_void_p),
        ("path_offsets", ctypes.c_void_p),
        ("cap_paths", ctypes.c_int64),
        ("path_vertices", ctypes.c_void_p),
        ("cap_vertices", ctypes.c_int64),
        ("header", ctypes.c_void_p),
    ]


P_STATUS, P_PATHS, P_VERTICES = range(3)
P_SLOTS = 4

SIMPLIFY_BUNDLE, SIMPLIFY_CANCEL = 0x1, 0x2


class eg_graph_host(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("nmax", ctypes.c_int64),
        ("maxima", ctypes.c_void_p),
        ("max_values", ctypes.c_void_p),
        ("nsad", ctypes.c_int64),
        ("saddles", ctypes.c_void_p),
        ("sad_values", ctypes.c_void_p),
        ("arc_offsets", ctypes.c_void_p),
        ("arc_maxima", ctypes.c_void_p),
    ]

_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    L.eg_workspace_bytes.argtypes = [ctypes.c_int, i64p, ctypes.c_int64]
    L.eg_workspace_bytes.restype = ctypes.c_size_t
    for name in ("eg_build", "eg_build_noalloc", "eg_classify", "eg_label", "eg_arcs"):
        fn = getattr(L, name)
        fn.argtypes = [vp, ctypes.c_int, i64p, vp, ctypes.POINTER(eg_out)]
        fn.restype = ctypes.c_int
    L.eg_build_streamed.argtypes = [vp, vp, ctypes.c_int, i64p, ctypes.c_int64, vp, vp, vp, ctypes.c_int64,
                                    ctypes.POINTER(eg_out)]
    L.eg_build_streamed.restype = ctypes.c_int
    L.eg_noalloc_scratch_bytes.argtypes = []
    L.eg_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.eg_paths.argtypes = [vp, ctypes.c_int, i64p, vp, ctypes.POINTER(eg_out), ctypes.POINTER(eg_paths_out)]
    L.eg_paths.restype = ctypes.c_int
    L.eg_simplify.argtypes = [ctypes.POINTER(eg_graph_host), ctypes.c_uint32, ctypes.c_double, vp, vp, vp, vp, vp,
                              vp, ctypes.POINTER(ctypes.c_int64)]
    L.eg_simplify.restype = ctypes.c_int
    L.eg_batch_plan_bytes.argtypes = [ctypes.c_int]
    L.eg_batch_plan_bytes.restype = ctypes.c_size_t
    L.eg_batch_workspace_bytes.argtypes = [ctypes.c_int, vp, vp, vp]
    L.eg_batch_workspace_bytes.restype = ctypes.c_size_t
    L.eg_batch_plan.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t]
    L.eg_batch_plan.restype = ctypes.c_int
    L.eg_build_batched.argtypes = [vp, vp]
    L.eg_build_batched.restype = ctypes.c_int
    L.eg_status_string.argtypes = [ctypes.c_int]
    L.eg_status_string.restype = ctypes.c_char_p
    L.eg_order_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int64]
    L.eg_order_workspace_bytes.restype = ctypes.c_size_t
    L.eg_order_field.argtypes = [ctypes.c_int, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
    L.eg_order_field.restype = ctypes.c_int
    L.eg_link_table.argtypes = [ctypes.c_int, vp, vp]
    L.eg_link_table.restype = ctypes.c_int
    _lib = L
    return L


def status_string(status: int) -> str:
    try:
        return lib().eg_status_string(int(status)).decode()
    except RuntimeError:
        return "?"


def _dims(shape):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return arr


def workspace_bytes(shape, cap_sad: int) -> int:
    return int(lib().eg_workspace_bytes(len(shape), _dims(shape), cap_sad))


def link_table(ndim: int):
    """Host-only neighbour table of the library: (offsets[k, ndim], adjacency):
    adjacency[j] is a Python int whose bit l is set iff rows j and l are
    adjacent."""
    import numpy as np

    k = lib().eg_link_table(ndim, None, None)
    if k < 0:
        raise EGError(EG_ERR_ARG, f"ndim={ndim}")
    words = (k + 63) // 64
    off = np.zeros((k, ndim), dtype=np.int8)
    raw = np.zeros(k * words, dtype=np.uint64)
    lib().eg_link_table(ndim, off.ctypes.data_as(ctypes.c_void_p), raw.ctypes.data_as(ctypes.c_void_p))
    # one Python int per row (rows of a 6D grid need two words)
    adj = [sum(int(raw[j * words + w]) << (64 * w) for w in range(words)) for j in range(k)]
    return off, adj


def default_caps(n: int, ndim: int) -> dict:
    """Starting capacities; the library reports exact needs if they are short."""
    sad = min(n, max(4096, n // (8 if ndim <= 3 else 4)))
    return {"cap_max": min(n, max(4096, n // 16)), "cap_sad": sad, "cap_arc": 3 * sad}


@dataclass
class EGResult:
    labels: torch.Tensor
    maxima: torch.Tensor
    saddles: torch.Tensor
    saddle_beta: torch.Tensor
    arc_offsets: torch.Tensor
    arc_maxima: torch.Tensor
    ptr: torch.Tensor | None
    passes: int
    counts: dict = dc_field(default_factory=dict)


@dataclass
class EGPaths:
    """Gradient-path geometry: saddle i owns paths pair_offsets[i] ..
    pair_offsets[i+1]; path k is vertices[path_offsets[k] .. path_offsets[k+1]]
    = saddle, rep, ..., maximum."""
    pair_offsets: torch.Tensor
    path_offsets: torch.Tensor
    vertices: torch.Tensor


# eg_dtype codes of the sample types eg_order_field accepts
DTYPES = {torch.float32: 0, torch.float64: 1, torch.int8: 2, torch.uint8: 3, torch.int16: 4, torch.uint16: 5,
          torch.int32: 6, torch.uint32: 7, torch.int64: 8, torch.uint64: 9}


def order_workspace_bytes(dtype: torch.dtype, n: int) -> int:
    if dtype not in DTYPES:
        raise EGError(EG_ERR_ARG, f"unsupported sample type {dtype}")
    return int(lib().eg_order_workspace_bytes(DTYPES[dtype], int(n)))


class Order:
    """Buffers of eg_order_field for fields of one type and size: the float32
    order surrogate and the sort workspace, allocated once."""

    def __init__(self, dtype: torch.dtype, n: int, device):
        self.dtype, self.n = dtype, int(n)
        self.out = torch.empty(self.n, dtype=torch.float32, device=device)
        self.ws_bytes = order_workspace_bytes(dtype, self.n)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device) if self.ws_bytes else None

    def launch(self, field: torch.Tensor, stream=None) -> torch.Tensor:
        """Queue eg_order_field on ``stream``; returns the surrogate (flat)."""
        if field.dtype != self.dtype or field.numel() != self.n or not field.is_cuda or not field.is_contiguous():
            raise EGError(EG_ERR_ARG, "field does not match this Order's type and size")
        s = stream if stream is not None else torch.cuda.current_stream(field.device)
        ws = ((self.ws.data_ptr() + 255) & ~255) if self.ws is not None else None
        st = lib().eg_order_field(DTYPES[self.dtype], ctypes.c_void_p(field.data_ptr()), self.n,
                                  ctypes.c_void_p(self.out.data_ptr()), ws, self.ws_bytes,
                                  ctypes.c_void_p(s.cuda_stream))
        if st != EG_OK:
            raise EGError(st, "eg_order_field")
        return self.out


def order_field(field: torch.Tensor, stream=None) -> torch.Tensor:
    """Float32 field with the same simulated-perturbation order as ``field``
    (any eg_dtype), in ``field``'s shape."""
    field = field.contiguous()
    return Order(field.dtype, field.numel(), field.device).launch(field, stream).view(field.shape)


class Builder:
    """Device buffers for repeated extremum-graph builds of one grid shape.

    ``launch(field)`` queues the work on the current stream and returns at
    once; ``finish()`` synchronises, reads the device header and returns an
    ``EGResult`` of views into the buffers (valid until the next launch).

    With ``noalloc=True`` no workspace is allocated and whole builds go
    through ``eg_build_noalloc`` (the library's fixed per-device scratch).
    """

    def __init__(self, shape, minima: bool = False, want_ptr: bool = False, device=None, tuning: int = 0,
                 noalloc: bool = False, **caps):
        self.shape = tuple(int(s) for s in shape)
        if not 1 <= len(self.shape) <= EG_MAX_NDIM:
            raise EGError(EG_ERR_ARG, f"ndim={len(self.shape)}")
        self.n = 1
        for s in self.shape:
            self.n *= s
        self.minima = minima
        self.want_ptr = want_ptr
        self.tuning = int(tuning)
        self.noalloc = bool(noalloc)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        c = default_caps(self.n, len(self.shape))
        c.update({k: int(v) for k, v in caps.items() if v is not None})
        self._alloc(c)

    def _alloc(self, caps):
        dev = self.device
        self.caps = dict(caps)
        i32 = dict(dtype=torch.int32, device=dev)
        self.labels = torch.empty(self.n, **i32)
        self.ptr = torch.empty(self.n, **i32) if self.want_ptr else None
        self.maxima = torch.empty(max(1, caps["cap_max"]), **i32)
        self.saddles = torch.empty(max(1, caps["cap_sad"]), **i32)
        self.beta = torch.empty(max(1, caps["cap_sad"]), **i32)
        self.offsets = torch.empty(caps["cap_sad"] + 1, **i32)
        self.arcs = torch.empty(max(1, caps["cap_arc"]), **i32)
        self.header = torch.zeros(H_SLOTS, **i32)
        ws = workspace_bytes(self.shape, caps["cap_sad"])
        if ws == 0:
            raise EGError(EG_ERR_ARG, f"workspace query failed for {self.shape} {caps}")
        if self.noalloc:
            self.ws, aligned, ws = None, None, 0
        else:
            self.ws = torch.empty(ws + 256, dtype=torch.uint8, device=dev)
            aligned = (self.ws.data_ptr() + 255) & ~255
        o = eg_out()
        o.flags = EG_MINIMA if self.minima else 0
        o.labels = self.labels.data_ptr()
        o.ptr = self.ptr.data_ptr() if self.ptr is not None else None
        o.maxima = self.maxima.data_ptr()
        o.cap_max = caps["cap_max"]
        o.saddles = self.saddles.data_ptr()
        o.saddle_beta = self.beta.data_ptr()
        o.arc_offsets = self.offsets.data_ptr()
        o.cap_sad = caps["cap_sad"]
        o.arc_maxima = self.arcs.data_ptr()
        o.cap_arc = caps["cap_arc"]
        o.workspace = aligned
        o.ws_bytes = ws
        o.header = self.header.data_ptr()
        o.tuning = self.tuning
        self.out = o
        self._dims = _dims(self.shape)

    def _float_field(self, field: torch.Tensor, s) -> torch.Tensor:
        """``field`` itself for float32, else its order surrogate (queued on s)."""
        if not field.is_cuda or not field.is_contiguous():
            raise EGError(EG_ERR_ARG, "field must be a contiguous device tensor")
        if field.numel() != self.n:
            raise EGError(EG_ERR_ARG, f"field has {field.numel()} values, builder expects {self.n}")
        if field.dtype == torch.float32:
            return field
        if field.dtype not in DTYPES:
            raise EGError(EG_ERR_ARG, f"unsupported sample type {field.dtype}")
        o = getattr(self, "_order", None)
        if o is None or o.dtype != field.dtype:
            o = self._order = Order(field.dtype, self.n, self.device)
        return o.launch(field, s)

    def launch(self, field: torch.Tensor, stream=None, stage: str = "all"):
        """Queue the whole path (``stage="all"``, eg_build) or one stage
        (``"classify"``, ``"label"``, ``"arcs"``) on ``stream`` (default: the
        current stream).  Fields of other sample types than float32 are first
        replaced by their order surrogate (eg_order_field)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        field = self._float_field(field, s)
        if self.noalloc and stage != "all":
            raise EGError(EG_ERR_ARG, "a no-alloc builder runs whole builds only")
        fn = {"all": lib().eg_build_noalloc if self.noalloc else lib().eg_build, "classify": lib().eg_classify,
              "label": lib().eg_label, "arcs": lib().eg_arcs}[stage]
        st = fn(ctypes.c_void_p(field.data_ptr()), len(self.shape), self._dims,
                ctypes.c_void_p(s.cuda_stream), ctypes.byref(self.out))
        if st != EG_OK:
            raise EGError(st)
        self._stream = s

    def launch_streamed(self, host: torch.Tensor, slab_planes: int, stream=None, copy_stream=None):
        """Queue eg_build_streamed: ``host`` (float32, pinned, this builder's
        shape) is copied to the builder's device field slab by slab on
        ``copy_stream`` while ``stream`` classifies the slabs that have
        landed.  Returns the device field."""
        if host.is_cuda or host.dtype != torch.float32 or not host.is_contiguous() or host.numel() != self.n:
            raise EGError(EG_ERR_ARG, "host field must be a contiguous float32 CPU tensor of the builder's shape")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        cs = getattr(self, "_copy_stream", None) if copy_stream is None else copy_stream
        if cs is None:
            cs = self._copy_stream = torch.cuda.Stream(device=self.device)
        if getattr(self, "field_dev", None) is None:
            self.field_dev = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        nslabs = -(-self.shape[0] // max(1, int(slab_planes)))
        evs = getattr(self, "_slab_events", [])
        while len(evs) < nslabs + 1:
            ev = torch.cuda.Event()
            ev.record(s)  # creates the event; the library records it again on the copy stream
            evs.append(ev)
        self._slab_events = evs
        handles = (ctypes.c_void_p * len(evs))(*[ev.cuda_event for ev in evs])
        st = lib().eg_build_streamed(ctypes.c_void_p(host.data_ptr()), ctypes.c_void_p(self.field_dev.data_ptr()),
                                     len(self.shape), self._dims, int(slab_planes), ctypes.c_void_p(s.cuda_stream),
                                     ctypes.c_void_p(cs.cuda_stream), handles, len(evs), ctypes.byref(self.out))
        if st != EG_OK:
            raise EGError(st, "eg_build_streamed")
        self._stream = s
        return self.field_dev

    def header_values(self):
        return [int(x) for x in self.header.cpu().tolist()]

    def finish(self, check: bool = True) -> EGResult:
        self._stream.synchronize()
        h = self.header_values()
        if check and h[H_STATUS] != EG_OK:
            raise EGError(h[H_STATUS], f"header={h}")
        nmax, nsad, narc = h[H_NMAX], h[H_NSAD], h[H_NARC]
        return EGResult(
            labels=self.labels.view(self.shape),
            maxima=self.maxima[:nmax],
            saddles=self.saddles[:nsad],
            saddle_beta=self.beta[:nsad],
            arc_offsets=self.offsets[:nsad + 1],
            arc_maxima=self.arcs[:max(narc, 0)],
            ptr=self.ptr.view(self.shape) if self.ptr is not None else None,
            passes=h[H_PASSES],
            counts={"maxima": nmax, "saddles": nsad, "arcs": narc, "pairs": h[H_NPAIRS], "exits": h[H_EXITS]},
        )

    def grow(self, h):
        """Reallocate with capacities large enough for the header's counts."""
        c = dict(self.caps)
        if h[H_NMAX] > c["cap_max"]:
            c["cap_max"] = h[H_NMAX]
        if h[H_NSAD] > c["cap_sad"]:
            c["cap_sad"] = h[H_NSAD]
        if h[H_NARC] > c["cap_arc"]:
            c["cap_arc"] = h[H_NARC]
        if h[H_NARC] < 0:
            # the arcs of the saddles past the old capacity were not counted
            c["cap_arc"] = max(c["cap_arc"], 3 * c["cap_sad"])
        self._alloc(c)

    def _alloc_paths(self, cap_paths: int, cap_vertices: int):
        i32 = dict(dtype=torch.int32, device=self.device)
        self.p_pair = torch.empty(self.caps["cap_sad"] + 1, **i32)
        self.p_off = torch.empty(cap_paths + 1, **i32)
        self.p_verts = torch.empty(max(1, cap_vertices), **i32)
        self.p_header = torch.zeros(P_SLOTS, **i32)
        po = eg_paths_out()
        po.pair_offsets = self.p_pair.data_ptr()
        po.path_offsets = self.p_off.data_ptr()
        po.cap_paths = cap_paths
        po.path_vertices = self.p_verts.data_ptr()
        po.cap_vertices = cap_vertices
        po.header = self.p_header.data_ptr()
        self.pout = po
        self.pcaps = (cap_paths, cap_vertices)

    def launch_paths(self, field: torch.Tensor, stream=None):
        """Queue eg_paths after a build of `field` on the same stream."""
        if self.ptr is None:
            raise EGError(EG_ERR_ARG, "paths need the steepest-ascent pointers: Builder(..., want_ptr=True)")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        field = self._float_field(field, s)
        st = lib().eg_paths(ctypes.c_void_p(field.data_ptr()), len(self.shape), self._dims,
                            ctypes.c_void_p(s.cuda_stream), ctypes.byref(self.out), ctypes.byref(self.pout))
        if st != EG_OK:
            raise EGError(st, "eg_paths")
        self._stream = s

    def paths(self, field: torch.Tensor, max_retries: int = 4) -> EGPaths:
        """Gradient-path geometry of the last build of `field` (run() first),
        growing the path buffers while the library reports a shortfall."""
        h = self.header_values()
        npairs = max(0, h[H_NPAIRS])
        if getattr(self, "pcaps", None) is None or self.pcaps[0] < npairs or self.p_pair.numel() < self.caps["cap_sad"] + 1:
            self._alloc_paths(max(1, npairs), max(64, 32 * npairs))
        for _ in range(max_retries + 1):
            self.launch_paths(field)
            self._stream.synchronize()
            ph = [int(x) for x in self.p_header.cpu().tolist()]
            if ph[P_STATUS] == EG_ERR_CAPACITY and h[H_NSAD] <= self.caps["cap_sad"]:
                self._alloc_paths(max(self.pcaps[0], ph[P_PATHS]), max(self.pcaps[1], ph[P_VERTICES]))
                continue
            if ph[P_STATUS] != EG_OK:
                raise EGError(ph[P_STATUS], f"paths header={ph}")
            nsad, npaths, nverts = h[H_NSAD], ph[P_PATHS], ph[P_VERTICES]
            return EGPaths(self.p_pair[:nsad + 1], self.p_off[:npaths + 1], self.p_verts[:nverts])
        raise EGError(EG_ERR_CAPACITY, "path capacity retries exhausted")

    def run(self, field: torch.Tensor, max_retries: int = 4) -> EGResult:
        """launch + finish, growing the buffers while the library reports a
        capacity shortfall."""
        for _ in range(max_retries + 1):
            self.launch(field)
            self._stream.synchronize()
            h = self.header_values()
            if h[H_STATUS] == EG_ERR_CAPACITY:
                self.grow(h)
                continue
            return self.finish()
        raise EGError(EG_ERR_CAPACITY, "capacity retries exhausted")

    def run_streamed(self, host: torch.Tensor, slab_planes: int, max_retries: int = 4) -> EGResult:
        """launch_streamed + finish, growing the buffers while the library
        reports a capacity shortfall (the field is copied again)."""
        for _ in range(max_retries + 1):
            self.launch_streamed(host, slab_planes)
            self._stream.synchronize()
            h = self.header_values()
            if h[H_STATUS] == EG_ERR_CAPACITY:
                self.grow(h)
                continue
            return self.finish()
        raise EGError(EG_ERR_CAPACITY, "capacity retries exhausted")


def build_streamed(host: torch.Tensor, slab_planes: int = 32, minima: bool = False, want_ptr: bool = False,
                   device=None, tuning: int = 0, **caps) -> EGResult:
    """Extremum graph of a host-resident float32 field (2D or 3D; pinned memory
    for the copy to overlap), copied slab by slab while earlier slabs are
    classified (eg_build_streamed)."""
    b = Builder(host.shape, minima=minima, want_ptr=want_ptr, device=device, tuning=tuning, **caps)
    return b.run_streamed(host.contiguous(), slab_planes)


class BatchBuilder:
    """Extremum graphs of many 2D/3D fields with one batched launch sequence.

    ``builders`` are per-field ``Builder`` objects (they own each field's
    output buffers and workspace); ``plan(fields)`` validates the batch,
    writes the plan on the host and copies it into the batch workspace on the
    current stream; ``launch()`` queues ``eg_build_batched``; ``finish()``
    synchronises and returns one ``EGResult`` per field.  A plan stays valid
    while the same field tensors and buffers are used, so repeated launches
    (benchmarks, HIP graph replays) need no new plan.
    """

    def __init__(self, shapes, minima=False, device=None, caps=None, tuning: int = 0):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        caps = caps or [None] * len(shapes)
        mins = minima if isinstance(minima, (list, tuple)) else [minima] * len(shapes)
        self.builders = [Builder(sh, minima=mn, device=self.device, tuning=tuning, **(c or {}))
                         for sh, mn, c in zip(shapes, mins, caps)]
        self._plan_host = None
        self._fields = None
        self._ws = None

    @classmethod
    def from_builders(cls, builders, device=None, reuse=None):
        """A batch over existing per-field builders; ``reuse`` lends its batch
        workspace and pinned plan buffer (it must not be in flight)."""
        bb = cls.__new__(cls)
        bb.device = torch.device(device) if device is not None else builders[0].device
        bb.builders = list(builders)
        bb._plan_host = None
        bb._fields = None
        bb._ws = reuse._ws if reuse is not None else None
        bb._pinned = getattr(reuse, "_pinned", None) if reuse is not None else None
        return bb

    @property
    def count(self):
        return len(self.builders)

    def _arrays(self):
        n = self.count
        ndims = (ctypes.c_int * n)(*[len(b.shape) for b in self.builders])
        dims = (ctypes.c_int64 * (n * EG_MAX_NDIM))()
        for i, b in enumerate(self.builders):
            for j, d in enumerate(b.shape):
                dims[i * EG_MAX_NDIM + j] = d
        outs = (eg_out * n)(*[b.out for b in self.builders])
        return ndims, dims, outs

    def plan(self, fields, stream=None):
        """Fields of other sample types than float32 are planned through their
        order surrogates (eg_order_field, one buffer per builder), which every
        launch() recomputes before the batch."""
        if len(fields) != self.count:
            raise EGError(EG_ERR_ARG, "one field per builder")
        for f, b in zip(fields, self.builders):
            if f.dtype not in DTYPES or not f.is_cuda or not f.is_contiguous() or f.numel() != b.n:
                raise EGError(EG_ERR_ARG, "fields must be contiguous device tensors of the builders' shapes")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        flo = [b._float_field(f, s) for f, b in zip(fields, self.builders)]
        L = lib()
        ndims, dims, outs = self._arrays()
        wsb = int(L.eg_batch_workspace_bytes(self.count, ndims, dims, outs))
        if wsb == 0:
            raise EGError(EG_ERR_ARG, "batch workspace query failed")
        if self._ws is None or self._ws.numel() < wsb + 256:
            self._ws = torch.empty(wsb + 256, dtype=torch.uint8, device=self.device)
        base = (self._ws.data_ptr() + 255) & ~255
        pb = int(L.eg_batch_plan_bytes(self.count))
        pinned = getattr(self, "_pinned", None)
        if pinned is None or pinned.numel() < pb:
            pinned = torch.empty(max(pb, 1 << 16), dtype=torch.uint8, pin_memory=True)
            self._pinned = pinned
        host = pinned[:pb]
        fptrs = (ctypes.c_void_p * self.count)(*[f.data_ptr() for f in flo])
        st = L.eg_batch_plan(self.count, fptrs, ndims, dims, outs, ctypes.c_void_p(base), wsb,
                             ctypes.c_void_p(host.data_ptr()), pb)
        if st != EG_OK:
            raise EGError(st, "eg_batch_plan")
        off = base - self._ws.data_ptr()
        with torch.cuda.stream(s):
            self._ws[off:off + pb].copy_(host, non_blocking=True)
        self._plan_host = host
        self._fields = list(fields)
        self._stream = s
        return self

    def launch(self, stream=None):
        if self._plan_host is None:
            raise EGError(EG_ERR_ARG, "plan() first")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        # typed fields: refresh their order surrogates (the plan points at them)
        for f, b in zip(self._fields, self.builders):
            if f.dtype != torch.float32:
                b._order.launch(f, s)
        st = lib().eg_build_batched(ctypes.c_void_p(self._plan_host.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        if st != EG_OK:
            raise EGError(st, "eg_build_batched")
        self._stream = s
        for b in self.builders:
            b._stream = s

    def finish(self, check: bool = True):
        self._stream.synchronize()
        return [b.finish(check=check) for b in self.builders]

    def run(self, fields, max_retries: int = 4):
        """plan + launch + finish, growing per-field buffers on capacity errors."""
        for _ in range(max_retries + 1):
            self.plan(fields)
            self.launch()
            self._stream.synchronize()
            heads = [b.header_values() for b in self.builders]
            short = [i for i, h in enumerate(heads) if h[H_STATUS] == EG_ERR_CAPACITY]
            if short:
                for i in short:
                    self.builders[i].grow(heads[i])
                continue
            return self.finish()
        raise EGError(EG_ERR_CAPACITY, "capacity retries exhausted")


def build_batched(fields, minima=False, **kw):
    """Extremum graphs of a list of 2D/3D device tensors (float32, or any type of
    DTYPES through its order surrogate) in one batch."""
    bb = BatchBuilder([f.shape for f in fields], minima=minima, device=fields[0].device, **kw)
    return bb.run([f.contiguous() for f in fields])


def build_paths(field: torch.Tensor, minima: bool = False, tuning: int = 0, **caps):
    """Extremum graph and gradient-path geometry of ``field``: (EGResult, EGPaths)."""
    b = Builder(field.shape, minima=minima, want_ptr=True, device=field.device, tuning=tuning, **caps)
    field = field.contiguous()
    r = b.run(field)
    return r, b.paths(field)


def build(field: torch.Tensor, minima: bool = False, want_ptr: bool = False, tuning: int = 0,
          **caps) -> EGResult:
    """Extremum graph of ``field`` (device tensor, 1..6 axes; float32, or any
    other type of DTYPES through its order surrogate)."""
    b = Builder(field.shape, minima=minima, want_ptr=want_ptr, device=field.device, tuning=tuning, **caps)
    return b.run(field.contiguous())


def simplify_graph(maxima, max_values, saddles, sad_values, arc_offsets, arc_maxima, ops: int, threshold: float,
                   minima: bool = False) -> dict:
    """eg_simplify on host (numpy) arrays of one extremum graph: arc bundling
    and/or persistence-directed cancellation (ops = SIMPLIFY_BUNDLE |
    SIMPLIFY_CANCEL).  Returns the simplified arcs of every saddle (CSR, empty
    rows for removed saddles), the representative of every maximum, and the
    cancellations in order."""
    import numpy as np

    arr = {
        "maxima": np.ascontiguousarray(maxima, dtype=np.int32),
        "max_values": np.ascontiguousarray(max_values, dtype=np.float64),
        "saddles": np.ascontiguousarray(saddles, dtype=np.int32),
        "sad_values": np.ascontiguousarray(sad_values, dtype=np.float64),
        "arc_offsets": np.ascontiguousarray(arc_offsets, dtype=np.int32),
        "arc_maxima": np.ascontiguousarray(arc_maxima, dtype=np.int32),
    }
    g = eg_graph_host()
    g.flags = EG_MINIMA if minima else 0
    g.nmax = arr["maxima"].size
    g.nsad = arr["saddles"].size
    for k, a in arr.items():
        setattr(g, k, a.ctypes.data_as(ctypes.c_void_p))
    narc = int(arr["arc_offsets"][-1]) if arr["arc_offsets"].size else 0
    offs = np.zeros(g.nsad + 1, np.int32)
    arcs = np.zeros(max(1, narc), np.int32)
    rep = np.zeros(max(1, g.nmax), np.int32)
    ps, pm = np.zeros(max(1, narc), np.int32), np.zeros(max(1, narc), np.int32)
    pc = np.zeros(max(1, narc), np.float64)
    n = ctypes.c_int64(0)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    st = lib().eg_simplify(ctypes.byref(g), int(ops), float(threshold), p(offs), p(arcs), p(rep), p(ps), p(pm),
                           p(pc), ctypes.byref(n))
    if st != EG_OK:
        raise EGError(st, "eg_simplify")
    k = int(n.value)
    return {"arc_offsets": offs, "arc_maxima": arcs[:int(offs[-1])], "max_rep": rep[:g.nmax],
            "pair_saddle": ps[:k], "pair_max": pm[:k], "pair_cost": pc[:k]}


def simplify(result: "EGResult", field: "torch.Tensor", ops: int = SIMPLIFY_BUNDLE | SIMPLIFY_CANCEL,
             threshold: float = 0.0, minima: bool = False) -> dict:
    """Simplify the graph of an eg.build result of ``field``: the values at its
    critical points are gathered on the device, the graph operations run on
    the host (eg_simplify)."""
    flat = field.reshape(-1)
    unsigned = {torch.uint16: (torch.int16, np.uint16), torch.uint32: (torch.int32, np.uint32),
                torch.uint64: (torch.int64, np.uint64)}
    if flat.dtype in unsigned:  # gather the bits through the signed type of the same width
        signed, host = unsigned[flat.dtype]
        flat = flat.view(signed)
        mv = flat[result.maxima.long()].cpu().numpy().view(host).astype(np.float64)
        sv = flat[result.saddles.long()].cpu().numpy().view(host).astype(np.float64)
    else:
        mv = flat[result.maxima.long()].cpu().numpy().astype(np.float64)
        sv = flat[result.saddles.long()].cpu().numpy().astype(np.float64)
    return simplify_graph(result.maxima.cpu().numpy(), mv, result.saddles.cpu().numpy(), sv,
                          result.arc_offsets.cpu().numpy(), result.arc_maxima.cpu().numpy(), ops, threshold, minima)
