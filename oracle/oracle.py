"""Python face of the C oracle (``eg_oracle.c``).

TEST INFRASTRUCTURE ONLY: this module is the oracle.  Only ``tests/``, the
smoke entry point and the benchmark's CPU-baseline leg may import it.  It does
not import the GPU library and the GPU library does not import it.

``extremum_graph`` returns the whole extremum graph of an array (C order,
``shape[0]`` slowest) as a dict of numpy arrays.  Samples keep their own type
when it is float32, float64 or an 8- to 64-bit integer (the C code compares
them as such); any other array is converted to float32 first.

* ``ptr``         steepest-ascent target of every vertex (itself at maxima)
* ``beta``        number of upper-link components of every vertex (Table 1)
* ``labels``      maximum reached from every vertex (its descending manifold)
* ``maxima``      ascending ids with beta == 0
* ``saddles``     ascending ids with beta >= 2
* ``saddle_beta`` beta of each saddle
* ``arc_offsets`` / ``arc_maxima``  CSR: the sorted distinct maxima reached
  from the reps (highest vertex of each upper-link component) of each saddle

``minima=True`` computes the minimum graph (the same steps under the reversed
order).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_I64P = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    _lib = _bind(ctypes.CDLL(_build.LIB))
    return _lib


def use_library(path):
    """Point this module at another build of ``eg_oracle.c`` (the mutation
    tests compile deliberately broken copies); ``None`` restores the default.
    Returns the previous library handle."""
    global _lib
    prev = _lib
    _lib = None if path is None else _bind(ctypes.CDLL(path))
    return prev


def _bind(lib):
    vp = ctypes.c_void_p
    lib.ego_num_threads.restype = ctypes.c_int
    lib.ego_set_threads.argtypes = [ctypes.c_int]
    lib.ego_set_threads.restype = ctypes.c_int
    ci = ctypes.c_int
    lib.ego_neighbours.argtypes = [vp, ci, ctypes.c_int, vp, ctypes.c_int64, vp]
    lib.ego_neighbours.restype = ctypes.c_int
    lib.ego_vertex.argtypes = [vp, ci, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int64, vp, vp]
    lib.ego_vertex.restype = ctypes.c_int
    lib.ego_label_of.argtypes = [vp, ci, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int64]
    lib.ego_label_of.restype = ctypes.c_int64
    lib.ego_classify.argtypes = [vp, ci, ctypes.c_int, vp, ctypes.c_int, vp, vp]
    lib.ego_classify.restype = ctypes.c_int
    lib.ego_labels.argtypes = [vp, ctypes.c_int64, vp]
    lib.ego_labels.restype = ctypes.c_int
    lib.ego_arcs.argtypes = [vp, ci, ctypes.c_int, vp, ctypes.c_int, vp, vp, ctypes.c_int64,
                             vp, vp, ctypes.c_int64, vp]
    lib.ego_arcs.restype = ctypes.c_int
    lib.ego_paths.argtypes = [vp, ci, ctypes.c_int, vp, ctypes.c_int, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int64,
                              vp, ctypes.c_int64, vp, vp]
    lib.ego_paths.restype = ctypes.c_int
    return lib


class OracleError(RuntimeError):
    pass


# numpy type -> the C oracle's sample-type code
DTYPES = {np.dtype(np.float32): 0, np.dtype(np.float64): 1, np.dtype(np.int8): 2, np.dtype(np.uint8): 3,
          np.dtype(np.int16): 4, np.dtype(np.uint16): 5, np.dtype(np.int32): 6, np.dtype(np.uint32): 7,
          np.dtype(np.int64): 8, np.dtype(np.uint64): 9}


def _prep(f):
    f = np.asarray(f)
    if f.dtype.newbyteorder("=") not in DTYPES:
        f = f.astype(np.float32)
    f = np.ascontiguousarray(f, dtype=f.dtype.newbyteorder("="))
    if f.ndim < 1:
        raise OracleError("need at least one axis")
    dims = np.asarray(f.shape, dtype=np.int64)
    return f, dims, DTYPES[f.dtype]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().ego_num_threads())


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the
    previous count."""
    return int(_load().ego_set_threads(int(n)))


def neighbours(shape, v: int) -> np.ndarray:
    """Neighbour ids of vertex ``v`` (Alg. 1 applied to every offset)."""
    lib = _load()
    dims = np.asarray(shape, dtype=np.int64)
    dummy = np.zeros(1, dtype=np.float32)
    out = np.zeros(600, dtype=np.int64)
    k = lib.ego_neighbours(_p(dummy), 0, len(shape), _p(dims), int(v), _p(out))
    if k < 0:
        raise OracleError("bad vertex")
    return np.sort(out[:k])


def vertex(f, v: int, minima: bool = False):
    """(ptr, beta, reps) of one vertex; reps ascending."""
    lib = _load()
    f, dims, dt = _prep(f)
    p = np.zeros(1, dtype=np.int64)
    reps = np.zeros(600, dtype=np.int64)
    b = lib.ego_vertex(_p(f), dt, f.ndim, _p(dims), int(minima), int(v), _p(p), _p(reps))
    if b < 0:
        raise OracleError("bad vertex")
    return int(p[0]), int(b), reps[:b].copy()


def label_of(f, v: int, minima: bool = False) -> int:
    lib = _load()
    f, dims, dt = _prep(f)
    r = lib.ego_label_of(_p(f), dt, f.ndim, _p(dims), int(minima), int(v))
    if r < 0:
        raise OracleError("bad vertex")
    return int(r)


def classify(f, minima: bool = False):
    """Per-vertex (ptr, beta) as int32 arrays of f.size."""
    lib = _load()
    f, dims, dt = _prep(f)
    n = f.size
    if n >= 2 ** 31:
        raise OracleError("too many vertices")
    ptr = np.empty(n, dtype=np.int32)
    beta = np.empty(n, dtype=np.int32)
    st = lib.ego_classify(_p(f), dt, f.ndim, _p(dims), int(minima), _p(ptr), _p(beta))
    if st == 4:
        raise OracleError("NaN in field")
    if st != 0:
        raise OracleError(f"oracle status {st}")
    return ptr, beta


def labels_from_ptr(ptr: np.ndarray) -> np.ndarray:
    lib = _load()
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    lab = np.empty_like(ptr)
    st = lib.ego_labels(_p(ptr), ptr.size, _p(lab))
    if st != 0:
        raise OracleError(f"oracle status {st}")
    return lab


def arcs(f, labels: np.ndarray, saddles: np.ndarray, minima: bool = False):
    lib = _load()
    f, dims, dt = _prep(f)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    saddles = np.ascontiguousarray(saddles, dtype=np.int32)
    offsets = np.zeros(saddles.size + 1, dtype=np.int32)
    cap = max(16, 3 * saddles.size)
    while True:
        am = np.empty(cap, dtype=np.int32)
        n_arc = np.zeros(1, dtype=np.int64)
        st = lib.ego_arcs(_p(f), dt, f.ndim, _p(dims), int(minima), _p(labels), _p(saddles),
                          saddles.size, _p(offsets), _p(am), cap, _p(n_arc))
        if st == 5:
            cap = int(n_arc[0])
            continue
        if st != 0:
            raise OracleError(f"oracle status {st}")
        return offsets, am[: int(n_arc[0])].copy()


def paths(f, ptr: np.ndarray, saddles: np.ndarray, minima: bool = False):
    """Gradient-path geometry (Alg. 2): (pair_offsets, path_offsets, vertices).
    Saddle i owns paths pair_offsets[i] .. pair_offsets[i+1]; path k is
    vertices[path_offsets[k] .. path_offsets[k+1]] = s, rep, ..., maximum."""
    lib = _load()
    f, dims, dt = _prep(f)
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    saddles = np.ascontiguousarray(saddles, dtype=np.int32)
    pair_offsets = np.zeros(saddles.size + 1, dtype=np.int32)
    cap_p, cap_v = max(16, 3 * saddles.size), max(64, 64 * saddles.size)
    while True:
        po = np.zeros(cap_p + 1, dtype=np.int32)
        verts = np.empty(cap_v, dtype=np.int32)
        n_p = np.zeros(1, dtype=np.int64)
        n_v = np.zeros(1, dtype=np.int64)
        st = lib.ego_paths(_p(f), dt, f.ndim, _p(dims), int(minima), _p(ptr), _p(saddles), saddles.size,
                           _p(pair_offsets), _p(po), cap_p, _p(verts), cap_v, _p(n_p), _p(n_v))
        if st == 5:
            cap_p, cap_v = max(cap_p, int(n_p[0])), max(cap_v, int(n_v[0]))
            continue
        if st != 0:
            raise OracleError(f"oracle status {st}")
        return pair_offsets, po[: int(n_p[0]) + 1].copy(), verts[: int(n_v[0])].copy()


def extremum_graph(f, minima: bool = False) -> dict:
    f = _prep(f)[0]
    ptr, beta = classify(f, minima)
    labels = labels_from_ptr(ptr)
    maxima = np.flatnonzero(beta == 0).astype(np.int32)
    saddles = np.flatnonzero(beta >= 2).astype(np.int32)
    offsets, arc_maxima = arcs(f, labels, saddles, minima)
    return {
        "ptr": ptr,
        "beta": beta,
        "labels": labels,
        "maxima": maxima,
        "saddles": saddles,
        "saddle_beta": beta[saddles].astype(np.int32),
        "arc_offsets": offsets,
        "arc_maxima": arc_maxima,
    }
