"""GPU parity: the HIP path (through the C ABI) equals the CPU oracle,
element by element, on seeded inputs.  Integer and ordering work only, so
the bar is bit-exact for every output."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_02724_amd import workloads as W
from tests.gpu_util import KEYS, assert_same, gpu_graph

pytestmark = pytest.mark.gpu

SMALL = [(1,), (2,), (37,), (1, 1), (5, 1), (1, 7), (6, 7), (33, 65), (3, 1, 4), (5, 4, 3), (17, 9, 70),
         (3, 3, 2, 3), (6, 5, 7, 4), (2, 2, 2, 2, 2), (3, 4, 3, 2, 3), (5, 6, 4, 5, 3),
         (2, 2, 2, 2, 2, 2), (1, 3, 2, 1, 2, 3), (4, 3, 5, 3, 4, 3)]


@pytest.mark.parametrize("shape", SMALL, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", ["uniform", "ties", "normal"])
def test_small_grids(shape, kind):
    for seed in range(2):
        f = W.random_field(shape, 100 + seed, kind)
        for minima in (False, True):
            ctx = f"shape={shape} kind={kind} seed={seed} minima={minima}"
            print(ctx, flush=True)
            g = gpu_graph(f, minima)
            o = O.extremum_graph(f, minima)
            assert_same(g, o, KEYS + ["ptr"], ctx)


@pytest.mark.parametrize("minima", [False, True])
def test_config0_2d_256(minima):
    f = W.field_2d_256()
    assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], f"2d256 minima={minima}")


@pytest.mark.parametrize("shape,corr", [((64, 64, 64), 4.0), ((40, 72, 96), 3.0)])
def test_grf_3d(shape, corr):
    f = W.gaussian_random_field(shape, 5, corr_len=corr, workers=4)
    for minima in (False, True):
        assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], f"grf {shape}")


def test_gaussian_mixture_5d():
    f = W.gaussian_mixture((12, 11, 10, 9, 8), 2, n_gauss=16, noise=1e-4)
    assert_same(gpu_graph(f), O.extremum_graph(f), KEYS + ["ptr"], "5d")


def test_6d_mixture_white_noise_and_schwefel():
    """6D grids: 126 neighbours, 128-bit upper-link masks."""
    f = W.gaussian_mixture((10, 9, 8, 8, 7, 6), 3, n_gauss=8, noise=1e-3)
    for minima in (False, True):
        assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], f"6d mix minima={minima}")
    g = W.random_field((7,) * 6, 5, "uniform")
    want = O.extremum_graph(g)
    assert np.diff(want["arc_offsets"]).max() == 8  # a full eight-entry arc list
    assert_same(gpu_graph(g), want, KEYS + ["ptr"], "6d noise")
    s = W.schwefel((12,) * 6)  # exact ties from the symmetric formula
    assert_same(gpu_graph(s), O.extremum_graph(s), KEYS + ["ptr"], "6d schwefel")


def test_6d_saddle_with_twenty_arcs():
    from tests.test_oracle_pins import twenty_arc_saddle
    f, centre, ids = twenty_arc_saddle()
    for minima in (False, True):
        want = O.extremum_graph(f, minima)
        assert_same(gpu_graph(f, minima), want, KEYS + ["ptr"], f"twenty arcs minima={minima}")
    g = gpu_graph(f)
    i = int(np.searchsorted(g["saddles"], centre))
    assert list(g["arc_maxima"][g["arc_offsets"][i]:g["arc_offsets"][i + 1]]) == ids


def test_gaussian_mixture_4d():
    f = W.gaussian_mixture((14, 13, 12, 11), 6, n_gauss=8, noise=1e-3)
    for minima in (False, True):
        assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], "4d")


@pytest.mark.parametrize("shape", [(301, 20, 20, 40), (45, 16, 16, 16, 33), (21, 8, 8, 8, 8, 20)])
def test_slab_tiles_several_planes_per_block(shape):
    """4D-6D grids large enough that each block of the slab classification
    runs over several planes along axis 0 (4, 6 and 2), the last block over
    fewer (1, 3 and 1), with ragged tiles along the other axes; white noise
    with ties (about 12 % saddles), both graphs."""
    f = W.random_field(shape, 90 + len(shape), "ties5")
    for minima in (False, True):
        ctx = f"slab {shape} minima={minima}"
        print(ctx, flush=True)
        assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], ctx)


@pytest.mark.parametrize("shape", [(300,), (40, 50), (9, 10, 11), (4, 5, 6, 7), (3, 4, 5, 4, 3)])
def test_constant_and_ramp(shape):
    const = np.full(shape, 1.5, np.float32)
    assert_same(gpu_graph(const), O.extremum_graph(const), KEYS + ["ptr"], "const")
    assert_same(gpu_graph(const, True), O.extremum_graph(const, True), KEYS + ["ptr"], "const min")
    n = len(shape)
    ramp = np.indices(shape).sum(0).astype(np.float32)  # many ties, long paths
    assert_same(gpu_graph(ramp), O.extremum_graph(ramp), KEYS + ["ptr"], "ramp")


def test_long_paths_need_several_jump_passes():
    # a single monotone serpentine-free ramp: the path from vertex 0 is N-1 steps
    f = np.arange(200000, dtype=np.float32)
    g = gpu_graph(f)
    assert np.all(g["labels"] == f.size - 1)
    assert g["passes"] >= 3


def test_signed_zero_and_infinities():
    rng = np.random.default_rng(3)
    f = rng.choice(np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0], np.float32), size=(30, 31))
    for minima in (False, True):
        assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], "zeros/inf")


def test_denormals_keep_their_order():
    # subnormal values must compare exactly (no flush to zero on the GPU path)
    rng = np.random.default_rng(5)
    vals = np.array([1e-45, 2e-45, 1e-40, 3e-39, -1e-45, -1e-40, 0.0, -0.0], np.float32)
    for shape in [(33, 70), (9, 17, 66)]:
        f = rng.choice(vals, size=shape)
        for minima in (False, True):
            assert_same(gpu_graph(f, minima), O.extremum_graph(f, minima), KEYS + ["ptr"], f"denormals {shape}")


def test_nan_reported():
    from paper_2303_02724_amd import eg
    f = W.random_field((20, 20), 1)
    f[3, 4] = np.nan
    with pytest.raises(eg.EGError) as ei:
        gpu_graph(f)
    assert ei.value.status == eg.EG_ERR_NAN


def test_capacity_overflow_then_retry():
    import torch
    from paper_2303_02724_amd import eg
    f = W.random_field((40, 30, 20), 8, "uniform")
    t = torch.from_numpy(f).cuda()
    b = eg.Builder(f.shape, cap_max=3, cap_sad=5, cap_arc=2)
    b.launch(t)
    h = b.header_values() if b._stream.synchronize() is None else None
    assert h[eg.H_STATUS] == eg.EG_ERR_CAPACITY
    o = O.extremum_graph(f)
    assert h[eg.H_NMAX] == o["maxima"].size
    assert h[eg.H_NSAD] == o["saddles"].size
    r = b.run(t)
    got = {"labels": r.labels.reshape(-1).cpu().numpy(), "maxima": r.maxima.cpu().numpy(),
           "saddles": r.saddles.cpu().numpy(), "saddle_beta": r.saddle_beta.cpu().numpy(),
           "arc_offsets": r.arc_offsets.cpu().numpy(), "arc_maxima": r.arc_maxima.cpu().numpy()}
    assert_same(got, o, KEYS, "after retry")


def test_repeat_runs_are_identical():
    f = W.gaussian_random_field((48, 48, 48), 9, corr_len=3.0, workers=4)
    a = gpu_graph(f)
    for _ in range(3):
        b = gpu_graph(f)
        assert_same(b, a, KEYS + ["ptr"], "repeat")


def _result_np(r):
    return {"labels": r.labels.reshape(-1).cpu().numpy(), "maxima": r.maxima.cpu().numpy(),
            "saddles": r.saddles.cpu().numpy(), "saddle_beta": r.saddle_beta.cpu().numpy(),
            "arc_offsets": r.arc_offsets.cpu().numpy(), "arc_maxima": r.arc_maxima.cpu().numpy()}


def test_batched_equals_oracle_mixed_shapes_and_modes():
    import torch
    from paper_2303_02724_amd import eg
    shapes = [(64, 64), (1, 1), (5, 70), (33, 129, 17), (40, 30, 20), (130, 70), (3, 2, 1), (70, 9, 65)]
    fields = [W.gaussian_mixture(sh, 300 + i, n_gauss=4, noise=1e-3) if len(sh) == 2 else
              W.random_field(sh, 300 + i, "ties" if i % 2 else "uniform") for i, sh in enumerate(shapes)]
    mins = [i % 3 == 1 for i in range(len(shapes))]
    ts = [torch.from_numpy(f).cuda() for f in fields]
    bb = eg.BatchBuilder([f.shape for f in fields], minima=mins)
    res = bb.run(ts)
    for f, m, r in zip(fields, mins, res):
        assert_same(_result_np(r), O.extremum_graph(f, m), KEYS, f"batched {f.shape} minima={m}")


def test_batched_replay_and_capacity_retry():
    import torch
    from paper_2303_02724_amd import eg
    specs = W.batched_specs(count=12, side2=(40, 300), side3=(16, 48))
    fields = [W.batched_field(sp) for sp in specs]
    ts = [torch.from_numpy(f).cuda() for f in fields]
    # tiny capacities force a capacity report and a retry with grown buffers
    caps = [{"cap_max": 1, "cap_sad": 1, "cap_arc": 1} for _ in fields]
    bb = eg.BatchBuilder([f.shape for f in fields], caps=caps)
    res = bb.run(ts)
    want = [O.extremum_graph(f) for f in fields]
    for f, r, o in zip(fields, res, want):
        assert_same(_result_np(r), o, KEYS, f"batched retry {f.shape}")
    # replay the same plan twice more: identical results
    for _ in range(2):
        bb.launch()
        again = bb.finish()
        for f, r, o in zip(fields, again, want):
            assert_same(_result_np(r), o, KEYS, f"batched replay {f.shape}")


def _pinned(f):
    import torch
    t = torch.empty(f.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(f)))
    return t


def test_serving_results_equal_the_oracle():
    """Continuous batching with host-resident fields (copied to the device at
    admission): every request's result equals the oracle's graph of its
    field, exactly, for small 2D/3D fields and a 192^3 field, with exact and
    with tiny starting capacities (requests then grow and run again), and
    the server never holds more device memory than its budget."""
    import torch
    from paper_2303_02724_amd import eg, serving
    specs = W.batched_specs(count=6, side2=(40, 400), side3=(16, 64), meta_seed=11)
    host = [W.batched_field(sp) for sp in specs]
    host.append(W.gaussian_mixture((192, 192, 192), 17, n_gauss=8, noise=1e-3))
    big = len(host) - 1
    want = [O.extremum_graph(f) for f in host]
    fields = [_pinned(f) for f in host]
    rng = np.random.default_rng(1)
    t, reqs = 0.0, []
    for i in range(60):
        t += rng.exponential(1 / 2000.0)
        reqs.append((t, big if i % 15 == 7 else int(rng.integers(0, big))))
    caps = {f.shape: {"cap_max": max(1, len(w["maxima"])), "cap_sad": max(1, len(w["saddles"])),
                      "cap_arc": max(1, len(w["arc_maxima"]))} for f, w in zip(host, want)}
    budget = 3 * serving.footprint_of(host[big].shape, caps[host[big].shape])
    for caps_for, exact in ((lambda sh: caps[sh], True), (lambda sh: {"cap_max": 1, "cap_sad": 1,
                                                                       "cap_arc": 1}, False)):
        got = {}
        srv = serving.Server(hbm_budget=budget, max_slots=8, max_batch=4, lanes=2, caps_for=caps_for)
        st = srv.run(reqs, fields, on_done=lambda ri, b: got.__setitem__(ri, _result_np(b.finish())))
        print(f"exact={exact}: {st.summary()}", flush=True)
        assert len(got) == len(reqs)
        assert st.copied_bytes == sum(host[fi].nbytes for _, fi in reqs)  # every field crossed PCIe once
        if exact:
            assert st.peak_bytes <= budget  # admission respects the budget
            assert st.regrown == 0
        else:
            assert st.regrown > 0  # undersized requests grew and ran again
        for ri, (_, fi) in enumerate(reqs):
            assert_same(got[ri], want[fi], KEYS, f"request {ri} field {fi} {host[fi].shape}")
        del srv
        torch.cuda.empty_cache()


def test_serving_batches_a_large_field_alone_and_with_others():
    """Device-resident fields arriving together are launched as batches of up
    to max_batch: the 192^3 field is served inside a batch and, arriving on
    its own later, as a single request; every result equals the oracle."""
    import torch
    from paper_2303_02724_amd import serving
    specs = W.batched_specs(count=5, side2=(40, 300), side3=(16, 48), meta_seed=12)
    host = [W.batched_field(sp) for sp in specs]
    host.append(W.gaussian_mixture((192, 192, 192), 18, n_gauss=8, noise=1e-3))
    big = len(host) - 1
    want = [O.extremum_graph(f) for f in host]
    fields = [torch.from_numpy(f).cuda() for f in host]
    reqs = [(0.0, i) for i in (0, 1, big, 2, 3, 4, 0, 1)] + [(0.5, big)]
    caps = {f.shape: {"cap_max": max(1, len(w["maxima"])), "cap_sad": max(1, len(w["saddles"])),
                      "cap_arc": max(1, len(w["arc_maxima"]))} for f, w in zip(host, want)}
    got, sizes = {}, {}
    srv = serving.Server(max_slots=16, max_batch=4, lanes=2, caps_for=lambda sh: caps[sh])
    st = srv.run(reqs, fields, on_done=lambda ri, b: got.__setitem__(ri, _result_np(b.finish())))
    for d in st.done:
        sizes[d.index] = d.size
    assert sizes[2] > 1 and sizes[8] == 1, sizes
    for ri, (_, fi) in enumerate(reqs):
        assert_same(got[ri], want[fi], KEYS, f"request {ri} field {fi}")


def test_every_tuning_gives_identical_results():
    """Launch choices (tile shapes, links per label pass) never change the
    output: each one equals the oracle on the same field."""
    from paper_2303_02724_amd import eg, tune
    f3 = W.gaussian_random_field((37, 45, 130), 12, corr_len=3.0, workers=4)
    f2 = W.gaussian_mixture((150, 200), 13, n_gauss=6, noise=1e-3)
    for f in (f3, f2):
        want = O.extremum_graph(f)
        for tu in tune.candidates(f.ndim) + [eg.tuning(hops=16)]:
            assert_same(gpu_graph(f, tuning=tu), want, KEYS + ["ptr"], f"tuning {tu:#x} {f.shape}")


def test_batched_with_tuning():
    import torch
    from paper_2303_02724_amd import eg
    specs = W.batched_specs(count=5, side2=(40, 200), side3=(16, 40), meta_seed=21)
    fields = [W.batched_field(sp) for sp in specs]
    ts = [torch.from_numpy(f).cuda() for f in fields]
    bb = eg.BatchBuilder([f.shape for f in fields], tuning=eg.tuning(tile3=1, tile2=1, hops=32))
    for f, r in zip(fields, bb.run(ts)):
        assert_same(_result_np(r), O.extremum_graph(f), KEYS, f"batched tuned {f.shape}")


@pytest.mark.parametrize("shape", [(8, 8, 8, 8, 8), (12, 12, 12, 12), (40, 40, 40)])
def test_saddles_with_more_than_four_arcs(shape):
    """The arc kernels keep the four smallest distinct arcs of a saddle in
    registers and find any further ones by extra passes: white noise has
    saddles with five and six distinct arcs in 3D, 4D and 5D."""
    f = W.random_field(shape, 5, "uniform")
    for minima in (False, True):
        want = O.extremum_graph(f, minima)
        assert np.diff(want["arc_offsets"]).max() > 4  # the case is present
        assert_same(gpu_graph(f, minima), want, KEYS + ["ptr"], f"{shape} minima={minima}")


def test_batched_saddles_with_more_than_four_arcs():
    import torch
    from paper_2303_02724_amd import eg
    fields = [W.random_field((40, 40, 40), 5, "uniform"), W.random_field((300, 200), 6, "uniform")]
    ts = [torch.from_numpy(f).cuda() for f in fields]
    for minima in (False, True):
        res = eg.BatchBuilder([f.shape for f in fields], minima=minima).run(ts)
        for f, r in zip(fields, res):
            assert_same(_result_np(r), O.extremum_graph(f, minima), KEYS, f"batched {f.shape} minima={minima}")


def test_batched_graph_replays_match_eager():
    """eg_build_batched captured in a HIP graph: every replay, with other
    device work and synchronisation between replays, gives the eager result
    (the library clears its counters with kernels, never with memsets)."""
    import torch
    from paper_2303_02724_amd import eg
    specs = W.batched_specs(count=9, side2=(40, 260), side3=(16, 44), meta_seed=31)
    fields = [W.batched_field(sp) for sp in specs]
    ts = [torch.from_numpy(f).cuda() for f in fields]
    bb = eg.BatchBuilder([f.shape for f in fields])
    eager = [_result_np(r) for r in bb.run(ts)]  # sizes the buffers, plans
    want = [O.extremum_graph(f) for f in fields]
    for e, o, f in zip(eager, want, fields):
        assert_same(e, o, KEYS, f"eager {f.shape}")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bb.launch(stream=side)  # warm the capture stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bb.launch(stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        for b in bb.builders:  # scribble on every output between replays
            b.labels.fill_(-7)
            b.arcs.fill_(-7)
            b.header.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b, e, f in zip(bb.builders, eager, fields):
            assert_same(_result_np(b.finish()), e, KEYS, f"replay {rep} {f.shape}")


@pytest.mark.parametrize("shape", [(48, 40, 36), (23, 21, 19, 17), (30, 300)])
def test_single_field_graph_replays_match_eager(shape):
    """eg_build of one field captured in a HIP graph (3D tiles, the untiled
    4D path, 2D tiles): every replay, with the outputs scribbled over and
    synchronisation between replays, gives the eager result."""
    import torch
    from paper_2303_02724_amd import eg
    f = W.gaussian_mixture(shape, 41, n_gauss=6, noise=1e-3)
    t = torch.from_numpy(f).cuda()
    b = eg.Builder(f.shape, want_ptr=True)
    eager = _result_np(b.run(t))
    assert_same(eager, O.extremum_graph(f), KEYS, f"eager {shape}")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.launch(t, stream=side)  # warm the capture stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        b.launch(t, stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        b.labels.fill_(-7)
        b.arcs.fill_(-7)
        b.header.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        b._stream = torch.cuda.current_stream()
        assert_same(_result_np(b.finish()), eager, KEYS, f"replay {rep} {shape}")


def _gpu_paths(f, minima=False, **caps):
    import torch
    from paper_2303_02724_amd import eg
    t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
    r, p = eg.build_paths(t, minima=minima, **caps)
    return (r, p.pair_offsets.cpu().numpy(), p.path_offsets.cpu().numpy(), p.vertices.cpu().numpy())


def _assert_paths(f, minima, ctx="", **caps):
    want = O.extremum_graph(f, minima)
    wp = O.paths(f, want["ptr"], want["saddles"], minima)
    r, *got = _gpu_paths(f, minima, **caps)
    for a, b, name in zip(got, wp, ("pair_offsets", "path_offsets", "vertices")):
        if not np.array_equal(a, b):
            raise AssertionError(f"{ctx} minima={minima} {name}: gpu {a[:12]} oracle {b[:12]} "
                                 f"sizes {a.size} {b.size}")


@pytest.mark.parametrize("shape", [(40,), (17, 23), (9, 10, 11), (7, 6, 5, 4), (5, 4, 5, 3, 4), (4, 3, 3, 4, 3, 3),
                                   (1, 1), (3, 2, 1)])
@pytest.mark.parametrize("kind", ["uniform", "ties"])
def test_paths_equal_oracle(shape, kind):
    f = W.random_field(shape, 61, kind)
    for minima in (False, True):
        _assert_paths(f, minima, f"{shape} {kind}")


def test_paths_grf_and_mixtures():
    f = W.gaussian_random_field((40, 72, 96), 9, corr_len=4.0, workers=4)
    _assert_paths(f, False, "grf")
    _assert_paths(f, True, "grf")
    g = W.gaussian_mixture((256, 256), 0, n_gauss=8, noise=1e-3)
    _assert_paths(g, False, "2d256")


def test_paths_long_and_capacity_regrowth():
    # one path thousands of vertices long (a serpentine-free ramp with a
    # saddle), and starting capacities far too small
    x = np.arange(3000, dtype=np.float32)
    f = np.concatenate([x, x[::-1] - 0.5, x + 100.0]).astype(np.float32)
    _assert_paths(f, False, "1d ramps")
    g = W.random_field((30, 40), 62, "uniform")
    _assert_paths(g, False, "tiny caps", cap_max=1, cap_sad=1, cap_arc=1)


def test_paths_reject_pointers_of_another_field():
    """A pointer array that does not describe the field (here: every entry
    outside the grid) ends each walk at once and is reported, never followed."""
    import torch
    from paper_2303_02724_amd import eg
    f = W.random_field((20, 30), 63, "uniform")
    t = torch.from_numpy(f).cuda()
    b = eg.Builder(f.shape, want_ptr=True)
    b.run(t)
    b.paths(t)  # valid first
    b.ptr.fill_(f.size + 5)
    b.launch_paths(t)
    torch.cuda.synchronize()
    assert int(b.p_header[eg.P_STATUS].item()) == eg.EG_ERR_ARG


def test_simplify_gpu_graph_equals_reference():
    """eg.simplify on a GPU-built graph (values gathered on the device) equals
    the reference simplification of the oracle's graph."""
    import torch
    from oracle import simplify as S
    from paper_2303_02724_amd import eg
    f = W.gaussian_mixture((40, 36, 32), 12, n_gauss=6, noise=1e-3)
    t = torch.from_numpy(f).cuda()
    fv = f.reshape(-1)
    for minima in (False, True):
        r = eg.build(t, minima=minima)
        want = O.extremum_graph(f, minima)
        g = (want["maxima"], fv[want["maxima"]], want["saddles"], fv[want["saddles"]], want["arc_offsets"],
             want["arc_maxima"])
        thr = 0.05
        lib = eg.simplify(r, t, threshold=thr, minima=minima)
        sm, ss, rows, pairs = S.cancel(*g, thr, minima, keep=S.bundle(*g, minima=minima))
        assert [(int(i), int(want["maxima"][m])) for i, m in zip(lib["pair_saddle"], lib["pair_max"])] == \
            [(i, m) for i, m, _ in pairs]
        lo, la = lib["arc_offsets"], lib["arc_maxima"]
        assert {i: la[lo[i]:lo[i + 1]].tolist() for i in range(len(lo) - 1) if lo[i + 1] > lo[i]} == \
            dict(zip(ss, rows))


def test_batched_long_paths_several_passes():
    """Paths far longer than a tile and than the links one pass follows
    (16 here): the exit-list chains need several gated jump passes before the
    tile-ordered pass can finish every vertex of every field."""
    import torch
    from paper_2303_02724_amd import eg
    shapes = [(2, 100000), (300, 700), (40, 50, 60), (3, 70, 4000)]
    fields = [np.arange(int(np.prod(sh)), dtype=np.float32).reshape(sh) for sh in shapes]
    fields.append(W.gaussian_mixture((200, 300), 77, n_gauss=4, noise=1e-3))
    ts = [torch.from_numpy(f).cuda() for f in fields]
    bb = eg.BatchBuilder([f.shape for f in fields], tuning=eg.tuning(hops=16))
    res = bb.run(ts)
    for f, r in zip(fields, res):
        assert_same(_result_np(r), O.extremum_graph(f), KEYS, f"batched long {f.shape}")
    # the path of the first field leaves a tile thousands of times, so its
    # exit-list chain is longer than 16 * 16 links: at least three passes
    assert res[0].counts["exits"] > 16 * 16


def test_autotuner_records_a_choice(tmp_path):
    import torch
    from paper_2303_02724_amd import tune
    f = torch.from_numpy(W.gaussian_random_field((48, 48, 64), 14, corr_len=3.0, workers=4)).cuda()
    path = str(tmp_path / "tune.json")
    res = tune.tune(f, reps=2, path=path)
    assert res["tuning"] in res["times_ms"]
    assert tune.best(tuple(f.shape), path=path) == res["tuning"]
