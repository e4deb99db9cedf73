"""Pins for the CPU oracle: it is checked against things other than itself.

* golden worked examples computed by hand (tests/golden/*.json),
* the literal all-pairs brute force (oracle/brute.py) on tiny grids, n = 1..6,
* neighbour counts, link f-vectors and the 3D upper-link histogram,
* closed forms (constant, linear, concave quadratic, 1D peaks and valleys),
* the Banchoff / Euler sum, which holds for any field on a triangulated box,
* symmetries: minima graph = maxima graph of the flipped, negated field;
  rank invariance; singleton axes; axis permutation.

Every test here runs on the CPU.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import brute as B
from oracle import oracle as O
from paper_2303_02724_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ["ptr", "beta", "labels", "maxima", "saddles", "saddle_beta", "arc_offsets", "arc_maxima"]


def _same(a, b, keys=KEYS):
    for k in keys:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# ------------------------------------------------------------------ golden

@pytest.mark.parametrize("name", ["worked_1d.json", "worked_2d_3x3.json"])
def test_golden_worked_examples(name):
    g = _load(name)
    f = np.array(g["field"], dtype=np.float32).reshape(g["shape"])
    for mode in ("max", "min"):
        if mode not in g:
            continue
        want = g[mode]
        for impl in (O.extremum_graph, B.extremum_graph):
            got = impl(f, minima=(mode == "min"))
            _same(got, want, [k for k in KEYS if k in want])


def test_neighbour_counts_and_link_fvectors():
    g = _load("link_counts.json")
    for n in range(1, 7):
        shape = (3,) * n
        centre = (3 ** n - 1) // 2
        nb = O.neighbours(shape, centre)
        assert len(nb) == g["neighbours"][str(n)] == 2 * (2 ** n - 1)
        if n < 2:
            continue
        coords = [np.unravel_index(int(v), shape) for v in nb]
        # cliques of pairwise-adjacent link vertices, by size
        adj = {i: {j for j in range(len(nb)) if j != i and B.grid_adjacency(coords[i], coords[j])}
               for i in range(len(nb))}
        counts = [len(nb)]
        level = [(i,) for i in range(len(nb))]
        while True:
            nxt = [c + (j,) for c in level for j in adj[c[-1]] if j > c[-1]
                   and all(j in adj[x] for x in c)]
            if not nxt:
                break
            counts.append(len(nxt))
            level = nxt
        assert counts == g["fvector"][str(n)]
        euler = sum((-1) ** i * c for i, c in enumerate(counts))
        assert euler == (0 if n % 2 == 0 else 2)


def test_link_fvectors_follow_the_ordered_partition_rule():
    """The golden f-vectors equal (k+1)! S(n+1, k+1): the link faces of a vertex
    of the Freudenthal tessellation are the ordered partitions of {0..n}."""
    from math import factorial

    def stirling2(n, k):
        if n == k:
            return 1
        if k == 0 or k > n:
            return 0
        return k * stirling2(n - 1, k) + stirling2(n - 1, k - 1)

    g = _load("link_counts.json")
    for n in range(2, 7):
        assert g["fvector"][str(n)] == [factorial(j) * stirling2(n + 1, j) for j in range(2, n + 2)]


@pytest.mark.parametrize("shape", [(7,) * 6, (9, 8, 7, 6, 5, 4)])
def test_schwefel_6d_invariants(shape):
    """Schwefel samples (symmetric, so rich in exact ties) on 6D grids."""
    f = W.schwefel(shape)
    for minima in (False, True):
        check_invariants(f, O.extremum_graph(f, minima), minima)


def twenty_arc_saddle():
    """A 3^6 grid whose centre has an upper link of the 20 neighbours at
    offsets with exactly three +1 entries: no two of them are adjacent (their
    difference has both signs), each is a maximum, so the centre is a saddle
    with beta = 20 and 20 arcs.  Returns (field, centre, the 20 ids)."""
    shape = (3,) * 6
    f = np.zeros(shape, np.float32)
    c = (1,) * 6
    f[c] = 1.0
    ids = []
    for k, ones in enumerate(itertools.combinations(range(6), 3)):
        p = tuple(2 if i in ones else 1 for i in range(6))
        f[p] = 2.0 + 0.01 * k
        ids.append(int(np.ravel_multi_index(p, shape)))
    return f, int(np.ravel_multi_index(c, shape)), sorted(ids)


def test_6d_saddle_with_twenty_arcs():
    f, centre, ids = twenty_arc_saddle()
    g = O.extremum_graph(f)
    i = int(np.searchsorted(g["saddles"], centre))
    assert g["saddles"][i] == centre and g["saddle_beta"][i] == 20
    assert list(g["arc_maxima"][g["arc_offsets"][i]:g["arc_offsets"][i + 1]]) == ids


def test_beta_histogram_3d():
    g = _load("link_counts.json")["beta_histogram_3d"]
    nb = O.neighbours((3, 3, 3), 13)
    hist = {}
    for m in range(1 << 14):
        f = np.zeros(27, np.float32)
        f[13] = 0.5
        for j in range(14):
            if m >> j & 1:
                f[nb[j]] = 1.0
        _, b, _ = O.vertex(f.reshape(3, 3, 3), 13)
        hist[b] = hist.get(b, 0) + 1
    assert {str(k): v for k, v in hist.items()} == g


# ------------------------------------------------------------------ brute force

BRUTE_SHAPES = [(9,), (1,), (2,), (6, 7), (1, 5), (2, 2), (5, 4, 3), (2, 3, 4), (1, 3, 1),
                (3, 3, 2, 3), (2, 2, 2, 2), (3, 2, 3, 2, 2), (3, 3, 3, 3, 3), (2, 2, 2, 2, 2),
                (2, 2, 2, 2, 2, 2), (3, 2, 2, 3, 2, 2), (1, 2, 3, 1, 2, 2)]


@pytest.mark.parametrize("shape", BRUTE_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", ["uniform", "ties"])
def test_oracle_matches_brute(shape, kind):
    for seed in range(2):
        f = W.random_field(shape, seed + 17 * len(shape), kind)
        for minima in (False, True):
            a = O.extremum_graph(f, minima)
            b = B.extremum_graph(f, minima)
            _same(a, b)


def test_oracle_matches_brute_alg2_reps():
    f = W.random_field((4, 4, 3), 5, "ties")
    b = B.extremum_graph(f)
    for s, reps in b["reps"].items():
        _, beta, oreps = O.vertex(f, s)
        assert beta == len(reps)
        assert list(oreps) == reps


# ------------------------------------------------------------------ path geometry

def _brute_paths(b):
    """The brute force's gradient paths, flattened in the oracle's layout."""
    pair_offsets, path_offsets, verts = [0], [0], []
    for s in b["saddles"]:
        for p in b["paths"][int(s)]:
            verts += list(p)
            path_offsets.append(len(verts))
        pair_offsets.append(len(path_offsets) - 1)
    return (np.array(pair_offsets, np.int32), np.array(path_offsets, np.int32), np.array(verts, np.int32))


@pytest.mark.parametrize("shape", [(9,), (6, 7), (5, 4, 3), (3, 3, 2, 3)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", ["uniform", "ties"])
def test_paths_match_brute(shape, kind):
    """The brute force's gradient paths (each rep's path built from its
    target's, highest vertex first) equal the oracle's walks of the pointers,
    in the same order: saddles ascending, components by their smallest vertex
    id."""
    for seed in range(2):
        f = W.random_field(shape, seed + 31 * len(shape), kind)
        for minima in (False, True):
            g = O.extremum_graph(f, minima)
            got = O.paths(f, g["ptr"], g["saddles"], minima)
            want = _brute_paths(B.extremum_graph(f, minima))
            for a, b, name in zip(got, want, ("pair_offsets", "path_offsets", "vertices")):
                np.testing.assert_array_equal(a, b, err_msg=f"{shape} {kind} minima={minima} {name}")


def _above(f, a, b, minima):
    fa, fb = float(f.flat[a]), float(f.flat[b])
    return (fa > fb or (fa == fb and a > b)) if not minima else (fb > fa or (fb == fa and b > a))


@pytest.mark.parametrize("shape", [(64, 64), (24, 20, 16), (10, 9, 8, 7)], ids=lambda s: "x".join(map(str, s)))
def test_path_invariants(shape):
    """Every path starts at its saddle, steps between Freudenthal neighbours,
    rises strictly in the order, and ends at the maximum that labels its
    rep; a saddle has beta+ paths whose ends are exactly its arc row."""
    f = W.gaussian_mixture(shape, 41, n_gauss=6, noise=1e-3)
    for minima in (False, True):
        g = O.extremum_graph(f, minima)
        po, pth, vs = O.paths(f, g["ptr"], g["saddles"], minima)
        assert po[-1] == pth.size - 1 == int(g["saddle_beta"].sum())
        maxima = set(g["maxima"].tolist())
        for i, s in enumerate(g["saddles"]):
            ends = set()
            assert po[i + 1] - po[i] == g["saddle_beta"][i]
            for k in range(po[i], po[i + 1]):
                p = vs[pth[k]:pth[k + 1]]
                assert p[0] == s and len(p) >= 2
                for a, b in zip(p[:-1], p[1:]):
                    assert b in set(O.neighbours(shape, int(a)).tolist())
                    assert _above(f, int(b), int(a), minima)
                assert int(p[-1]) in maxima and g["labels"][p[1]] == p[-1]
                ends.add(int(p[-1]))
            row = g["arc_maxima"][g["arc_offsets"][i]:g["arc_offsets"][i + 1]]
            assert ends == set(row.tolist())


def test_nan_rejected():
    f = W.random_field((4, 4), 1)
    f[2, 3] = np.nan
    with pytest.raises(O.OracleError):
        O.extremum_graph(f)


def test_signed_zero_and_inf():
    # -0 and +0 compare equal, so the index decides; infinities order normally
    f = np.array([0.0, -0.0, 0.0, np.inf, -np.inf, 1.0], dtype=np.float32)
    g = O.extremum_graph(f)
    f2 = np.array([0.0, 0.0, 0.0, 3.0, -3.0, 1.0], dtype=np.float32)
    _same(g, O.extremum_graph(f2))


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("shape", [(17,), (6, 5), (4, 5, 3), (3, 4, 2, 3), (3, 2, 3, 2, 3)])
def test_constant_field(shape):
    f = np.full(shape, 0.25, np.float32)
    N = f.size
    g = O.extremum_graph(f)
    assert list(g["maxima"]) == [N - 1]
    assert g["saddles"].size == 0
    assert np.all(g["labels"] == N - 1)
    h = O.extremum_graph(f, minima=True)
    assert list(h["maxima"]) == [0]
    assert h["saddles"].size == 0
    assert np.all(h["labels"] == 0)


@pytest.mark.parametrize("shape", [(6, 5), (4, 5, 3), (3, 4, 2, 3), (3, 2, 3, 2, 3)])
def test_generic_linear_field(shape):
    n = len(shape)
    w = np.array([1.0 + 0.37 * i + 0.011 * i * i for i in range(n)])[::-1]
    c = np.indices(shape).reshape(n, -1).T
    f = (c @ w).reshape(shape).astype(np.float32)
    g = O.extremum_graph(f)
    assert list(g["maxima"]) == [f.size - 1]
    assert g["saddles"].size == 0
    h = O.extremum_graph(f, minima=True)
    assert list(h["maxima"]) == [0]
    assert h["saddles"].size == 0


@pytest.mark.parametrize("shape,p", [((9, 8), (3.3, 5.2)), ((7, 6, 5), (2.2, 4.4, 1.3)),
                                      ((5, 4, 5, 4), (1.4, 2.3, 3.1, 0.8))])
def test_concave_quadratic(shape, p):
    n = len(shape)
    c = np.indices(shape).reshape(n, -1).T.astype(np.float64)
    f = (-((c - np.array(p)) ** 2).sum(1)).reshape(shape).astype(np.float32)
    g = O.extremum_graph(f)
    peak = np.ravel_multi_index(tuple(int(round(x)) for x in p), shape)
    assert list(g["maxima"]) == [peak]
    assert g["saddles"].size == 0
    assert np.all(g["labels"] == peak)


def _peaks_1d(a):
    """1D closed form: maxima, saddles (both neighbours higher), and for each
    saddle the peaks reached by climbing left and right."""
    n = len(a)
    hi = lambda i, j: a[i] > a[j] or (a[i] == a[j] and i > j)  # noqa: E731
    maxima = [i for i in range(n) if all(hi(i, j) for j in (i - 1, i + 1) if 0 <= j < n)]
    saddles = [i for i in range(1, n - 1) if hi(i - 1, i) and hi(i + 1, i)]

    def climb(i, step):
        while 0 <= i + step < n and hi(i + step, i):
            i += step
        return i

    rows = [sorted({climb(s - 1, -1), climb(s + 1, +1)}) for s in saddles]
    return maxima, saddles, rows


@pytest.mark.parametrize("seed", range(6))
def test_1d_closed_form(seed):
    a = W.random_field((200,), seed, "uniform" if seed % 2 == 0 else "ties5")
    maxima, saddles, rows = _peaks_1d([float(x) for x in a])
    g = O.extremum_graph(a)
    assert list(g["maxima"]) == maxima
    assert list(g["saddles"]) == saddles
    got = [list(g["arc_maxima"][g["arc_offsets"][i]:g["arc_offsets"][i + 1]]) for i in range(len(saddles))]
    assert got == rows


# ------------------------------------------------------------------ Banchoff sum

def test_banchoff_2d_from_beta():
    """In 2D the upper link of a vertex is part of a hexagon (a path at the
    boundary), so chi(upper link) = beta+ except for an interior vertex whose
    whole link is upper (chi = 0).  The sum of 1 - chi over all vertices is the
    Euler characteristic of the rectangle, 1."""
    for seed, kind in [(0, "uniform"), (1, "ties"), (2, "uniform")]:
        f = W.random_field((23, 17), seed, kind)
        g = O.extremum_graph(f)
        lo = O.extremum_graph(f, minima=True)
        H, Wd = f.shape
        total = 0
        interior_min = set(int(m) for m in lo["maxima"])
        for v in range(f.size):
            y, x = divmod(v, Wd)
            interior = 0 < y < H - 1 and 0 < x < Wd - 1
            chi = 0 if (interior and v in interior_min) else int(g["beta"][v])
            total += 1 - chi
        assert total == 1


@pytest.mark.parametrize("shape", [(7, 6, 5), (4, 3, 4, 3), (3, 3, 2, 3, 2), (2, 3, 2, 2, 3, 2)])
def test_banchoff_nd(shape):
    """Sum over vertices of 1 - chi(upper link) = chi(box) = 1, with the upper
    link's faces counted as cliques of pairwise-adjacent upper neighbours (the
    Freudenthal complex is a flag complex)."""
    f = W.random_field(shape, 3, "ties")
    flat = f.reshape(-1)
    total = 0
    for v in range(f.size):
        nb = [int(u) for u in O.neighbours(shape, v)]
        up = [u for u in nb if (flat[u], u) > (flat[v], v)]
        coords = {u: np.unravel_index(u, shape) for u in up}
        adj = {u: {w for w in up if w != u and B.grid_adjacency(coords[u], coords[w])} for u in up}
        chi, level, sign = 0, [(u,) for u in up], 1
        while level:
            chi += sign * len(level)
            sign = -sign
            level = [c + (w,) for c in level for w in adj[c[-1]] if w > c[-1]
                     and all(w in adj[x] for x in c)]
        total += 1 - chi
    assert total == 1


# ------------------------------------------------------------------ symmetries

@pytest.mark.parametrize("shape", [(9, 7), (5, 4, 6), (3, 4, 3, 3), (3, 3, 2, 3, 3)])
def test_minima_graph_is_flipped_negated_maxima_graph(shape):
    """Flipping every axis maps index i to N-1-i and keeps the tessellation, so
    the minimum graph of f (reversed order) equals the maximum graph of the
    flipped, negated field with every id mapped through i -> N-1-i."""
    for kind in ("uniform", "ties"):
        f = W.random_field(shape, 7, kind)
        N = f.size
        g = -np.flip(f)
        lo = O.extremum_graph(f, minima=True)
        hi = O.extremum_graph(np.ascontiguousarray(g))
        m = lambda a: np.sort(N - 1 - np.asarray(a))  # noqa: E731
        assert np.array_equal(lo["maxima"], m(hi["maxima"]))
        assert np.array_equal(lo["saddles"], m(hi["saddles"]))
        assert np.array_equal(lo["labels"], (N - 1 - hi["labels"])[::-1])
        assert np.array_equal(lo["ptr"], (N - 1 - hi["ptr"])[::-1])
        rows_lo = {int(s): tuple(lo["arc_maxima"][lo["arc_offsets"][i]:lo["arc_offsets"][i + 1]])
                   for i, s in enumerate(lo["saddles"])}
        rows_hi = {N - 1 - int(s): tuple(sorted(N - 1 - hi["arc_maxima"][hi["arc_offsets"][i]:hi["arc_offsets"][i + 1]]))
                   for i, s in enumerate(hi["saddles"])}
        assert rows_lo == rows_hi


@pytest.mark.parametrize("shape", [(30, 21), (9, 8, 7), (5, 4, 5, 4)])
def test_rank_invariance(shape):
    for kind in ("uniform", "ties"):
        f = W.random_field(shape, 11, kind)
        flat = f.reshape(-1).astype(np.float64)
        order = np.lexsort((np.arange(flat.size), flat))
        rank = np.empty(flat.size, np.float32)
        rank[order] = np.arange(flat.size, dtype=np.float32)
        for minima in (False, True):
            _same(O.extremum_graph(f, minima), O.extremum_graph(rank.reshape(shape), minima))


def test_singleton_axes_collapse():
    f = W.random_field((11, 9), 4, "ties")
    base = O.extremum_graph(f)
    for shape in [(11, 9, 1), (1, 11, 9), (11, 1, 9), (1, 11, 1, 9, 1)]:
        _same(O.extremum_graph(f.reshape(shape)), base)


@pytest.mark.parametrize("shape,perm", [((6, 5, 4), (2, 0, 1)), ((6, 5, 4), (1, 2, 0)),
                                         ((4, 3, 5, 3), (3, 1, 0, 2))])
def test_axis_permutation(shape, perm):
    """The tessellation is invariant under permuting axes; with no ties the
    order is too, so the graph maps through the index permutation."""
    f = W.random_field(shape, 9, "uniform")
    g = np.ascontiguousarray(np.transpose(f, perm))
    a = O.extremum_graph(f)
    b = O.extremum_graph(g)
    idx = np.arange(f.size).reshape(shape)
    to_g = np.empty(f.size, np.int64)
    to_g[idx.reshape(-1)] = np.transpose(idx, perm).reshape(-1).argsort()
    # to_g[i] = index in g of the vertex that has index i in f
    assert np.array_equal(np.sort(to_g[a["maxima"]]), b["maxima"])
    assert np.array_equal(np.sort(to_g[a["saddles"]]), b["saddles"])
    assert np.array_equal(to_g[a["labels"]], b["labels"][to_g])
    assert np.array_equal(to_g[a["ptr"]], b["ptr"][to_g])


# ------------------------------------------------------------------ invariants

def check_invariants(f, g, minima=False):
    """Properties every correct extremum graph has, at any size."""
    shape = f.shape
    N = f.size
    flat = f.reshape(-1)
    lab, ptr, beta = g["labels"], g["ptr"], g["beta"]
    maxima = g["maxima"]
    ismax = np.zeros(N, bool)
    ismax[maxima] = True
    assert np.array_equal(np.flatnonzero(beta == 0), maxima)
    assert np.array_equal(np.flatnonzero(beta >= 2), g["saddles"])
    assert np.all(ismax[lab])
    assert np.array_equal(lab[lab], lab)
    assert np.array_equal(lab[ptr], lab)
    assert np.array_equal(ptr[maxima], maxima)
    assert np.unique(lab).size == maxima.size

    def above(a, b):
        fa, fb = flat[a], flat[b]
        if minima:
            return (fb > fa) | ((fb == fa) & (b > a))
        return (fa > fb) | ((fa == fb) & (a > b))

    v = np.arange(N)
    nonmax = ~ismax
    assert np.all(above(ptr[nonmax], v[nonmax]))
    assert np.all(above(lab[nonmax], v[nonmax]))
    offs, am = g["arc_offsets"], g["arc_maxima"]
    rows = np.diff(offs)
    assert np.all(rows >= 1) and np.all(rows <= g["saddle_beta"])
    assert np.all(ismax[am])
    sad_rep = np.repeat(g["saddles"], rows)
    assert np.all(above(am, sad_rep))
    for i in range(len(g["saddles"])):
        r = am[offs[i]:offs[i + 1]]
        assert np.all(np.diff(r) > 0)


@pytest.mark.parametrize("shape", [(64, 48), (20, 18, 16), (9, 8, 7, 6), (6, 5, 6, 5, 4), (5, 4, 5, 4, 4, 5)])
def test_invariants_on_gaussian_mixtures(shape):
    f = W.gaussian_mixture(shape, 5, n_gauss=6, noise=1e-3)
    for minima in (False, True):
        g = O.extremum_graph(f, minima)
        check_invariants(f, g, minima)


def test_sampled_queries_match_whole_field():
    f = W.gaussian_mixture((12, 11, 10), 8, n_gauss=5, noise=1e-3)
    g = O.extremum_graph(f)
    rng = np.random.default_rng(0)
    for v in rng.integers(0, f.size, 40):
        p, b, reps = O.vertex(f, int(v))
        assert p == g["ptr"][v] and b == g["beta"][v]
        assert O.label_of(f, int(v)) == g["labels"][v]


# ------------------------------------------------------------------ sample types

TYPED = W.TYPED


@pytest.mark.parametrize("dt", TYPED)
def test_typed_fields_match_brute(dt):
    """Every sample type the paper's input accepts (Sec. 4) is compared in its
    own type: the brute force compares Python ints / floats exactly."""
    for shape in [(23,), (6, 7), (4, 3, 4), (3, 2, 3, 3), (2, 3, 2, 2, 3)]:
        f = W.typed_field(shape, 5 + len(shape), dt)
        for minima in (False, True):
            _same(O.extremum_graph(f, minima), B.extremum_graph(f, minima))


@pytest.mark.parametrize("dt", TYPED)
def test_typed_fields_rank_invariance(dt):
    """The graph depends on the order only: a typed field and its float32 rank
    field (ranks by numpy's stable sort of the native values) agree."""
    for shape in [(40, 33), (12, 11, 10), (6, 5, 6, 5)]:
        f = W.typed_field(shape, 9, dt)
        flat = f.reshape(-1)
        if flat.dtype == np.float64:
            flat = np.where(flat == 0, 0.0, flat)  # -0 == +0 before the sort
        order = np.argsort(flat, kind="stable")
        rank = np.empty(flat.size, np.float32)
        rank[order] = np.arange(flat.size, dtype=np.float32)
        for minima in (False, True):
            _same(O.extremum_graph(f, minima), O.extremum_graph(rank.reshape(f.shape), minima))


def test_float64_nan_rejected():
    f = W.typed_field((5, 4), 1, "float64")
    f[1, 2] = np.nan
    with pytest.raises(O.OracleError):
        O.extremum_graph(f)
