"""Autotuner for the launch configuration of the extremum-graph library.

The library exposes launch choices that never change results (eg_out.tuning:
3D tile shape, 2D tile shape, links followed per label pass).  ``tune`` times
every candidate on a given field with HIP events on the launch stream and
records the fastest for the field's size class; ``best`` returns the recorded
choice (or the defaults).  The cache is a small JSON file keyed by
``ndim`` and the power-of-two size class of the vertex count.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import torch

from . import eg

DEFAULT_CACHE = os.environ.get("EG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "eg_tune.json"))

TILES3 = (0, 1, 2)   # 64x8x8, 64x4x16, 64x8x4
TILES2 = (0, 1)      # 64x32, 64x16
HOPS = (32, 64, 128)


def size_class(shape) -> str:
    n = 1
    for s in shape:
        n *= int(s)
    return f"{len(shape)}d_2^{max(0, int(math.log2(max(n, 1))))}"


def candidates(ndim: int):
    tiles = [(t, 0) for t in TILES3] if ndim == 3 else [(0, t) for t in TILES2] if ndim == 2 else [(0, 0)]
    return [eg.tuning(tile3=t3, tile2=t2, hops=h) for (t3, t2), h in itertools.product(tiles, HOPS)]


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def best(shape, path: str = DEFAULT_CACHE) -> int:
    """Recorded tuning for the size class of ``shape`` (0 = library defaults)."""
    return int(_load(path).get(size_class(shape), {}).get("tuning", 0))


def tune(field: torch.Tensor, minima: bool = False, reps: int = 5, path: str | None = DEFAULT_CACHE) -> dict:
    """Time every candidate launch configuration on ``field`` and record the
    fastest for its size class.  Returns {tuning: ms} and the choice."""
    s = torch.cuda.current_stream()
    times = {}
    ref = None
    for tu in candidates(field.dim()):
        b = eg.Builder(field.shape, minima=minima, tuning=tu, device=field.device)
        r = b.run(field)  # sizes buffers; also checks the status
        sig = (r.maxima.cpu().numpy().tobytes(), r.arc_maxima.cpu().numpy().tobytes(),
               r.labels.cpu().numpy().tobytes())
        if ref is None:
            ref = sig
        elif sig != ref:
            raise RuntimeError(f"tuning {tu:#x} changed the result")
        b.launch(field, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            b.launch(field, stream=s)
        e1.record(s)
        e1.synchronize()
        times[tu] = e0.elapsed_time(e1) / reps
    choice = min(times, key=times.get)
    if path:
        data = _load(path)
        data[size_class(field.shape)] = {"tuning": choice, "ms": times[choice],
                                         "default_ms": times.get(eg.tuning(hops=64), None)}
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return {"times_ms": times, "tuning": choice}
