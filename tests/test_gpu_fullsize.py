"""GPU parity at the full benchmark sizes, in the launch configurations the
benchmark times: every output of the HIP path equals the oracle's, bit for
bit, on the whole field (the oracle takes seconds per field on the host's
cores), plus the invariants every extremum graph has.

* 512^3 Gaussian random field: both graphs, every launch configuration the
  autotuner chooses from (3D tile shape x links per label pass);
* 32^5 Gaussian mixture (maxima): every pass length;
* 16^6 Schwefel samples (maxima): every pass length;
* the 512^3 field built from pinned host memory in 32-plane slabs;
* the 256 batched fields, in one batch with exact-fit capacities as the
  benchmark runs them.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2303_02724_amd import eg, tune
from paper_2303_02724_amd import workloads as W
from tests.gpu_util import KEYS, assert_same

pytestmark = pytest.mark.gpu


def _graph(r):
    out = {
        "labels": r.labels.reshape(-1).cpu().numpy(),
        "maxima": r.maxima.cpu().numpy(),
        "saddles": r.saddles.cpu().numpy(),
        "saddle_beta": r.saddle_beta.cpu().numpy(),
        "arc_offsets": r.arc_offsets.cpu().numpy(),
        "arc_maxima": r.arc_maxima.cpu().numpy(),
    }
    if r.ptr is not None:
        out["ptr"] = r.ptr.reshape(-1).cpu().numpy()
    return out


def _invariants(f, g, minima):
    """Every vertex carries a maximum as its label; labels are fixed points and
    agree along each pointer; pointers rise; label count = maxima count; arc
    rows are ascending, distinct, non-empty, at most beta long and end at
    maxima above their saddle."""
    flat = f.reshape(-1)
    lab, ptr, mx = g["labels"], g["ptr"], g["maxima"]
    ismax = np.zeros(flat.size, bool)
    ismax[mx] = True
    assert np.all(ismax[lab]) and np.array_equal(lab[lab], lab) and np.array_equal(lab[ptr], lab)
    assert np.array_equal(ptr[mx], mx) and np.unique(lab).size == mx.size

    def above(a, b):
        fa, fb = flat[a], flat[b]
        if minima:
            return (fb > fa) | ((fb == fa) & (b > a))
        return (fa > fb) | ((fa == fb) & (a > b))

    v = np.flatnonzero(~ismax)
    assert np.all(above(ptr[v], v))
    offs, am = g["arc_offsets"], g["arc_maxima"]
    rows = np.diff(offs)
    assert np.all(rows >= 1) and np.all(rows <= g["saddle_beta"])
    assert np.all(ismax[am]) and np.all(above(am, np.repeat(g["saddles"], rows)))
    assert np.all(np.diff(mx) > 0) and np.all(np.diff(g["saddles"]) > 0)


def test_full_512_grf_every_launch_configuration():
    f = W.field_3d_grf(512, seed=1)
    t = torch.from_numpy(f).cuda()
    for minima in (False, True):
        want = O.extremum_graph(f, minima)
        configs = tune.candidates(3) if not minima else [eg.tuning(hops=64)]
        for tu in configs:
            ctx = f"512^3 minima={minima} tuning={tu:#x}"
            print(ctx, flush=True)
            g = _graph(eg.build(t, minima=minima, want_ptr=True, tuning=tu))
            assert_same(g, want, KEYS + ["ptr"], ctx)
        _invariants(f, g, minima)


def test_full_5d_32_every_pass_length():
    f = W.field_5d_32(seed=2)
    t = torch.from_numpy(f).cuda()
    want = O.extremum_graph(f)
    for tu in tune.candidates(5):
        ctx = f"32^5 tuning={tu:#x}"
        print(ctx, flush=True)
        g = _graph(eg.build(t, want_ptr=True, tuning=tu))
        assert_same(g, want, KEYS + ["ptr"], ctx)
    _invariants(f, g, False)


def test_full_6d_16_schwefel_every_pass_length():
    """The 6D benchmark grid at its full size (16^6 = 16.8 M vertices): the
    symmetric Schwefel samples have many exact ties and saddles joining many
    maxima."""
    f = W.field_6d(16)
    t = torch.from_numpy(f).cuda()
    want = O.extremum_graph(f)
    for tu in tune.candidates(6):
        ctx = f"16^6 tuning={tu:#x}"
        print(ctx, flush=True)
        g = _graph(eg.build(t, want_ptr=True, tuning=tu))
        assert_same(g, want, KEYS + ["ptr"], ctx)
    _invariants(f, g, False)


def test_full_512_streamed():
    """The streamed build of the 512^3 field from pinned host memory, in the
    slab height the benchmark times (32 planes), equals the oracle."""
    f = W.field_3d_grf(512, seed=1)
    host = torch.from_numpy(f).pin_memory()
    want = O.extremum_graph(f)
    g = _graph(eg.build_streamed(host, 32, want_ptr=True))
    assert_same(g, want, KEYS + ["ptr"], "512^3 streamed, 32-plane slabs")


def test_full_batched_256_fields():
    specs = W.batched_specs()
    fields = [W.batched_field(sp) for sp in specs]
    ts = [torch.from_numpy(f).cuda() for f in fields]
    bb = eg.BatchBuilder([f.shape for f in fields])
    bb.run(ts)
    caps = []
    for b in bb.builders:
        h = b.header_values()
        caps.append({"cap_max": max(1, h[eg.H_NMAX]), "cap_sad": max(1, h[eg.H_NSAD]),
                     "cap_arc": max(1, h[eg.H_NARC])})
    bb = eg.BatchBuilder([f.shape for f in fields], caps=caps)
    res = bb.run(ts)
    for i, (f, r) in enumerate(zip(fields, res)):
        ctx = f"batched field {i} shape={f.shape}"
        if i % 32 == 0:
            print(ctx, flush=True)
        assert_same(_graph(r), O.extremum_graph(f), KEYS, ctx)
