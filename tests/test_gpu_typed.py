"""GPU parity for the other sample types (int8..int64, uint8..uint64,
float64): eg.build on a typed device tensor (its order surrogate from
eg_order_field, then the float32 path) equals the oracle, which compares the
samples in their own type.  Bit-exact, like every output of the path."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2303_02724_amd import eg
from paper_2303_02724_amd import workloads as W
from tests.gpu_util import KEYS, assert_same

pytestmark = pytest.mark.gpu

RANKED = ["float64", "int32", "uint32", "int64", "uint64"]


def _dev(f):
    return torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0")


def typed_graph(f, minima=False, **caps):
    r = eg.build(_dev(f), minima=minima, want_ptr=True, **caps)
    return {
        "labels": r.labels.reshape(-1).cpu().numpy(),
        "ptr": r.ptr.reshape(-1).cpu().numpy(),
        "maxima": r.maxima.cpu().numpy(),
        "saddles": r.saddles.cpu().numpy(),
        "saddle_beta": r.saddle_beta.cpu().numpy(),
        "arc_offsets": r.arc_offsets.cpu().numpy(),
        "arc_maxima": r.arc_maxima.cpu().numpy(),
    }


SHAPES = [(1,), (37,), (6, 7), (33, 65), (5, 4, 3), (17, 9, 70), (6, 5, 7, 4), (3, 4, 3, 2, 3)]


@pytest.mark.parametrize("dt", W.TYPED)
def test_typed_small_grids(dt):
    for shape in SHAPES:
        f = W.typed_field(shape, 40 + len(shape), dt)
        for minima in (False, True):
            ctx = f"dtype={dt} shape={shape} minima={minima}"
            print(ctx, flush=True)
            assert_same(typed_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], ctx)


@pytest.mark.parametrize("dt", RANKED)
def test_typed_several_sort_blocks(dt):
    # 88560 samples: six sort blocks, a ragged last tile
    f = W.typed_field((48, 45, 41), 7, dt)
    for minima in (False, True):
        ctx = f"dtype={dt} minima={minima}"
        print(ctx, flush=True)
        assert_same(typed_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], ctx)


def _check_surrogate(f, ctx):
    """(out[u], u) and (f[u], u) sort the same way (numpy's stable sort; -0
    folded into +0 first); ranked types leave no ties in out."""
    print(ctx, flush=True)
    out = eg.order_field(_dev(f)).cpu().numpy().reshape(-1)
    flat = f.reshape(-1)
    if flat.dtype.kind == "f":
        flat = np.where(flat == 0, np.zeros_like(flat), flat)
    want = np.argsort(flat, kind="stable")
    got = np.argsort(out, kind="stable")
    bad = np.flatnonzero(want != got)
    assert bad.size == 0, f"{ctx}: {bad.size} positions differ, first {bad[:5]}"
    if f.dtype.itemsize >= 4 and f.dtype != np.float32:
        assert np.unique(out).size == out.size, ctx


def test_order_surrogate_large_and_every_pass():
    rng = np.random.Generator(np.random.PCG64(77))
    n = 3_000_001  # 184 sort blocks
    cases = {
        "f64 normal": rng.standard_normal(n),
        "f64 clustered": W.typed_field((n,), 78, "float64"),
        "i32 full range": rng.integers(-2 ** 31, 2 ** 31, size=n, dtype=np.int64).astype(np.int32),
        "u32 two values": np.where(rng.random(n) < 0.5, 2 ** 31 + 5, 7).astype(np.uint32),
        "i64 clustered": W.typed_field((n,), 79, "int64"),
        "u64 full range": rng.integers(0, 2 ** 63, size=n, dtype=np.uint64) * np.uint64(2) + np.uint64(1),
        "i64 one pass": rng.integers(-60, 60, size=n).astype(np.int64),  # 7-bit key range
        "i64 constant": np.full(n, -3, np.int64),  # no pass runs
        "u8": rng.integers(0, 256, size=n).astype(np.uint8),
        "i16": rng.integers(-2 ** 15, 2 ** 15, size=n).astype(np.int16),
    }
    for name, f in cases.items():
        _check_surrogate(f, name)


def test_typed_nan_reported():
    f = W.typed_field((20, 30), 3, "float64")
    f[4, 5] = np.nan
    with pytest.raises(eg.EGError) as e:
        typed_graph(f)
    assert e.value.status == eg.EG_ERR_NAN


def test_typed_paths_and_simplify():
    from oracle import simplify as S
    f = W.typed_field((30, 28, 26), 11, "int32")
    for minima in (False, True):
        r, p = eg.build_paths(_dev(f), minima=minima)
        want = O.extremum_graph(f, minima)
        wp = O.paths(f, want["ptr"], want["saddles"], minima)
        for a, b, name in zip((p.pair_offsets, p.path_offsets, p.vertices), wp,
                              ("pair_offsets", "path_offsets", "vertices")):
            assert np.array_equal(a.cpu().numpy(), b), f"{name} minima={minima}"
        fv = f.reshape(-1).astype(np.float64)
        g = (want["maxima"], fv[want["maxima"]], want["saddles"], fv[want["saddles"]], want["arc_offsets"],
             want["arc_maxima"])
        thr = 2.0 ** 30
        lib = eg.simplify(r, _dev(f), threshold=thr, minima=minima)
        _, ss, rows, pairs = S.cancel(*g, thr, minima, keep=S.bundle(*g, minima=minima))
        assert [(int(i), int(want["maxima"][m])) for i, m in zip(lib["pair_saddle"], lib["pair_max"])] == \
            [(i, m) for i, m, _ in pairs]
        lo, la = lib["arc_offsets"], lib["arc_maxima"]
        assert {i: la[lo[i]:lo[i + 1]].tolist() for i in range(len(lo) - 1) if lo[i + 1] > lo[i]} == \
            dict(zip(ss, rows))


def test_typed_fields_in_a_batch():
    """A batch mixing sample types: each field goes through its order
    surrogate, recomputed at every launch; results equal the oracle's."""
    dts = ["int16", "float64", "uint32", "int64", "uint8", "int32"]
    shapes = [(50, 61), (18, 17, 19), (33, 70), (12, 23, 16), (64, 9), (21, 20, 22)]
    fields = [W.typed_field(sh, 300 + i, dt) for i, (sh, dt) in enumerate(zip(shapes, dts))]
    ts = [_dev(f) for f in fields]
    bb = eg.BatchBuilder([f.shape for f in fields], minima=[False, True, False, True, False, True])
    res = bb.run(ts)
    for i, (f, r) in enumerate(zip(fields, res)):
        minima = i % 2 == 1
        got = {"labels": r.labels.reshape(-1).cpu().numpy(), "maxima": r.maxima.cpu().numpy(),
               "saddles": r.saddles.cpu().numpy(), "saddle_beta": r.saddle_beta.cpu().numpy(),
               "arc_offsets": r.arc_offsets.cpu().numpy(), "arc_maxima": r.arc_maxima.cpu().numpy()}
        assert_same(got, O.extremum_graph(f, minima), KEYS, f"field {i} {dts[i]} {f.shape}")
    # new values in the same tensors: a relaunch of the same plan refreshes the surrogates
    for i, t in enumerate(ts):
        g = W.typed_field(fields[i].shape, 400 + i, dts[i])
        t.copy_(_dev(g))
        fields[i] = g
    bb.launch()
    for i, (f, r) in enumerate(zip(fields, bb.finish())):
        minima = i % 2 == 1
        assert np.array_equal(r.labels.reshape(-1).cpu().numpy(), O.extremum_graph(f, minima)["labels"]), i
