"""Seeded synthetic scalar fields on regular grids.

These generators are the only code shared by the GPU path, the CPU oracle and
the benchmark: they produce input samples and nothing else.  None of the
extremum-graph arithmetic (adjacency, ordering, link components, labels) lives
here.

The paper measures real volumes (Open SciVis, Table 3) and samples of the
Schwefel function (Table 4).  Those datasets are not available, so seeded
synthetic fields of the same shapes stand in for them:

* ``gaussian_mixture``: a sum of isotropic Gaussian bumps plus uniform noise on
  the unit cube, sampled at ``j_i / (d_i - 1)`` along every axis.  It stands in
  for the small smooth volumes (2D 256^2, 5D 32^5 like Schwefel 5D 32^5).
* ``gaussian_random_field``: white noise smoothed by a Gaussian spectral
  filter, standing in for the 512^3-class volumes.
* ``batched_fields`` / ``serving_stream``: many fields of uneven sizes.

Every field is computed in float64 from numpy ``Generator(PCG64(seed))`` and
rounded to float32 once (round to nearest even).
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _axis_coords(d: int) -> np.ndarray:
    if d == 1:
        return np.zeros(1, dtype=np.float64)
    return np.arange(d, dtype=np.float64) / float(d - 1)


def gaussian_mixture(shape, seed: int, n_gauss: int = 8, sigma=(0.03, 0.1),
                     amp=(0.5, 1.0), noise: float = 1e-3) -> np.ndarray:
    """Sum of ``n_gauss`` isotropic Gaussians plus uniform noise, as float32.

    Draw order: centres (U[0,1)^n per bump), then sigma, then amplitudes, then
    the noise field (U[0, noise) per vertex).  Bump g contributes
    ``a_g * exp(-|x - c_g|^2 / (2 sigma_g^2))``.
    """
    shape = tuple(int(s) for s in shape)
    n = len(shape)
    rng = _rng(seed)
    centres = rng.random((n_gauss, n))
    sig = rng.uniform(sigma[0], sigma[1], size=n_gauss)
    amps = rng.uniform(amp[0], amp[1], size=n_gauss)
    out = np.zeros(shape, dtype=np.float64)
    axes = [_axis_coords(d) for d in shape]
    for g in range(n_gauss):
        # separable evaluation: the product of 1D factors, broadcast over the grid
        term = np.asarray(amps[g], dtype=np.float64)
        for i in range(n):
            fac = np.exp(-((axes[i] - centres[g, i]) ** 2) / (2.0 * sig[g] ** 2))
            bshape = [1] * n
            bshape[i] = shape[i]
            term = term * fac.reshape(bshape)
        out += term
    if noise > 0:
        out += rng.uniform(0.0, noise, size=shape)
    return out.astype(np.float32)


def gaussian_random_field(shape, seed: int, corr_len: float = 8.0,
                          workers: int | None = None) -> np.ndarray:
    """Gaussian random field: N(0,1) white noise times the spectral kernel
    ``exp(-2 pi^2 s^2 |k|^2)`` (k in cycles per voxel, s = ``corr_len`` voxels,
    i.e. a spatial Gaussian blur of standard deviation s), normalised to mean 0
    and standard deviation 1 in float64, rounded to float32.  The filter is
    periodic but the grid is not (no wrap-around adjacency is implied)."""
    import scipy.fft as sfft

    shape = tuple(int(s) for s in shape)
    if workers is None:
        workers = max(1, min(16, os.cpu_count() or 1))
    rng = _rng(seed)
    noise = rng.standard_normal(shape)
    spec = sfft.rfftn(noise, workers=workers)
    del noise
    k2 = None
    for i, d in enumerate(shape):
        k = sfft.rfftfreq(d) if i == len(shape) - 1 else sfft.fftfreq(d)
        bshape = [1] * len(shape)
        bshape[i] = k.shape[0]
        term = (k ** 2).reshape(bshape)
        k2 = term if k2 is None else k2 + term
    spec *= np.exp(-2.0 * np.pi ** 2 * corr_len ** 2 * k2)
    field = sfft.irfftn(spec, s=shape, workers=workers)
    del spec
    field -= field.mean()
    field /= field.std()
    return field.astype(np.float32)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------- workloads

def field_2d_256(seed: int = 0) -> np.ndarray:
    """2D 256x256: 8 Gaussians + U[0,1e-3) noise (max and min graphs)."""
    return gaussian_mixture((256, 256), seed, n_gauss=8, noise=1e-3)


def field_3d_grf(side: int = 512, seed: int = 1) -> np.ndarray:
    """3D side^3 Gaussian random field, correlation length 8 voxels."""
    return gaussian_random_field((side, side, side), seed, corr_len=8.0)


def schwefel(shape) -> np.ndarray:
    """The Schwefel function 418.9829 n - sum_i x_i sin(sqrt|x_i|) sampled on
    x_i = -500 + 1000 j_i / (d_i - 1), in float64, rounded to float32 once.
    The paper's higher-dimensional timings (Table 4) use samples of it; the
    published formula is evaluated here.  On a cube grid it is symmetric under
    axis permutations, so equal values (resolved by the index tie-break) are
    common."""
    shape = tuple(int(s) for s in shape)
    n = len(shape)
    out = np.full(shape, 418.9829 * n, dtype=np.float64)
    for i, d in enumerate(shape):
        x = -500.0 + 1000.0 * _axis_coords(d) if d > 1 else np.zeros(1)
        term = x * np.sin(np.sqrt(np.abs(x)))
        out -= term.reshape((1,) * i + (d,) + (1,) * (n - i - 1))
    return out.astype(np.float32)


def field_6d(side: int = 16) -> np.ndarray:
    """6D side^6 Schwefel samples (Table 4's 6D grids are 16^6, 24^6, 32^6)."""
    return schwefel((side,) * 6)


def field_5d_32(seed: int = 2, side: int = 32) -> np.ndarray:
    """5D side^5: 16 Gaussians + U[0,1e-4) noise (maxima graph)."""
    return gaussian_mixture((side,) * 5, seed, n_gauss=16, noise=1e-4)


@dataclass
class FieldSpec:
    shape: tuple
    seed: int


def batched_specs(count: int = 256, meta_seed: int = 3,
                  side2=(64, 2048), side3=(32, 192)) -> list[FieldSpec]:
    """Shapes of the batched workload: ndim 2 or 3 with probability 1/2 each,
    every side independently uniform on the closed integer range; field i
    uses value seed 1000 + i."""
    rng = _rng(meta_seed)
    specs = []
    for i in range(count):
        if rng.random() < 0.5:
            shape = tuple(int(s) for s in rng.integers(side2[0], side2[1] + 1, size=2))
        else:
            shape = tuple(int(s) for s in rng.integers(side3[0], side3[1] + 1, size=3))
        specs.append(FieldSpec(shape, 1000 + i))
    return specs


def batched_field(spec: FieldSpec) -> np.ndarray:
    return gaussian_mixture(spec.shape, spec.seed, n_gauss=8, noise=1e-3)


@dataclass
class Request:
    arrival_s: float
    spec: FieldSpec


def serving_stream(n_requests: int = 2000, rate_hz: float = 200.0, seed: int = 4,
                   big_side: int = 384, p_big: float = 0.1,
                   side2=(64, 2048), side3=(32, 192)) -> list[Request]:
    """Poisson arrivals at ``rate_hz``; each request is a batched-workload
    shape, or a ``big_side``^3 field with probability ``p_big``."""
    rng = _rng(seed)
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        if rng.random() < p_big:
            shape = (big_side,) * 3
        elif rng.random() < 0.5:
            shape = tuple(int(s) for s in rng.integers(side2[0], side2[1] + 1, size=2))
        else:
            shape = tuple(int(s) for s in rng.integers(side3[0], side3[1] + 1, size=3))
        reqs.append(Request(t, FieldSpec(shape, 20000 + i)))
    return reqs


def random_field(shape, seed: int, kind: str = "uniform") -> np.ndarray:
    """Small test fields: ``uniform`` U[0,1); ``ties`` integers {0,1,2};
    ``ties5`` integers {0..4}; ``normal`` N(0,1)."""
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    if kind == "uniform":
        a = rng.random(shape)
    elif kind == "ties":
        a = rng.integers(0, 3, size=shape).astype(np.float64)
    elif kind == "ties5":
        a = rng.integers(0, 5, size=shape).astype(np.float64)
    elif kind == "normal":
        a = rng.standard_normal(shape)
    else:
        raise ValueError(kind)
    return a.astype(np.float32)


TYPED = ("float64", "int8", "uint8", "int16", "uint16", "int32", "uint32", "int64", "uint64")


def typed_field(shape, seed: int, dtype: str) -> np.ndarray:
    """Fields of other sample types, drawn so that a comparison made in a
    narrower or differently signed type would change the order:

    * float64: small integers plus multiples of 2^-40 (equal after rounding to
      float32, distinct in float64), with -0, +0 and infinities mixed in;
    * 8- and 16-bit integers: a handful of values drawn over the whole range
      plus its two ends (many ties);
    * 32-bit: a few clusters spread over the whole range (both sides of 2^31
      for uint32, of 0 for int32), members 0..3 apart (equal in float32);
    * 64-bit: the same with clusters spread over the whole 64-bit range
      (members equal in float64).
    """
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    dt = np.dtype(dtype)
    if dt == np.float64:
        a = rng.integers(0, 4, size=n).astype(np.float64) + rng.integers(0, 4, size=n) * 2.0 ** -40
        special = rng.random(n)
        a[special < 0.04] = -0.0
        a[(special >= 0.04) & (special < 0.08)] = 0.0
        a[(special >= 0.08) & (special < 0.10)] = np.inf
        a[(special >= 0.10) & (special < 0.12)] = -np.inf
        return a.reshape(shape)
    info = np.iinfo(dt)
    if dt.itemsize <= 2:
        vals = np.concatenate([rng.integers(int(info.min), int(info.max) + 1, size=5, dtype=np.int64),
                               [int(info.min), int(info.max)]])
        return vals[rng.integers(0, vals.size, size=n)].astype(dt).reshape(shape)
    # cluster centres anywhere in the range (kept 4 away from its ends), then small offsets
    lo, hi = int(info.min), int(info.max) - 4
    centres = [int(x) for x in rng.integers(0, 2 ** 62, size=4)]
    span = hi - lo
    cs = [lo + (c * span) // (2 ** 62) for c in centres] + [lo, hi, (lo + hi) // 2]
    pick = rng.integers(0, len(cs), size=n)
    off = rng.integers(0, 4, size=n)
    out = np.empty(n, dtype=dt)
    for i in range(n):
        out[i] = cs[int(pick[i])] + int(off[i])
    return out.reshape(shape)
