"""Pins of the simplification reference (oracle/simplify.py, Sec. 3.5):
hand-worked graphs (simple saddles, multi-saddles whose cost is the gap to the
second-highest maximum, an order of cancellations that differs from the elder
rule), the 1D chain, persistence pairs equal to the textbook elder-rule
pairing of the superlevel sets on graphs whose saddles are all simple, and the
surviving maximum of every connected part of a multi-saddle graph."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import simplify as S
from paper_2303_02724_amd import workloads as W


def _graph(f, minima):
    g = O.extremum_graph(f, minima)
    fv = np.asarray(f, np.float32).reshape(-1)
    return (g["maxima"], fv[g["maxima"]], g["saddles"], fv[g["saddles"]], g["arc_offsets"], g["arc_maxima"])


def _hand(max_values, sad_values, rows):
    """A hand-made graph: maxima 0..M-1, saddles 100.. with the given rows."""
    maxima = np.arange(len(max_values), dtype=np.int32)
    saddles = np.arange(100, 100 + len(sad_values), dtype=np.int32)
    offs = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    arcs = np.array([m for r in rows for m in r], np.int32)
    return (maxima, np.asarray(max_values, np.float64), saddles, np.asarray(sad_values, np.float64), offs, arcs)


def test_hand_worked_bundling_and_cancellation():
    # maxima 0 (height 5) and 1 (height 4); three saddles joining them at
    # heights 1, 2, 3, and a saddle joining maximum 1 to maximum 2 (height 9)
    maxima = np.array([0, 1, 2], np.int32)
    mv = np.array([5.0, 4.0, 9.0], np.float32)
    saddles = np.array([10, 11, 12, 13], np.int32)
    sv = np.array([1.0, 2.0, 3.0, 3.5], np.float32)
    offs = np.array([0, 2, 4, 6, 8], np.int32)
    arcs = np.array([0, 1, 0, 1, 0, 1, 1, 2], np.int32)
    # bundling: the pair (0, 1) keeps saddle 12 (the highest), (1, 2) keeps 13
    assert S.bundle(maxima, mv, saddles, sv, offs, arcs) == [2, 3]
    # cancellation after bundling, threshold 1: saddle 13 joins maxima 1 (4)
    # and 2 (9) and costs 4 - 3.5 = 0.5, saddle 12 costs 4 - 3 = 1; 13 goes
    # first and merges maximum 1 into maximum 2; saddle 12 then joins 0 (5)
    # and 2 and costs 5 - 3 = 2 > 1: kept
    sm, ss, rows, pairs = S.cancel(maxima, mv, saddles, sv, offs, arcs, 1.0, keep=[2, 3])
    assert pairs == [(3, 1, 0.5)]
    assert sm == [0, 2] and ss == [2] and rows == [[0, 2]]
    # threshold 2: then saddle 12 merges maximum 0 into maximum 2
    sm, ss, rows, pairs = S.cancel(maxima, mv, saddles, sv, offs, arcs, 2.0, keep=[2, 3])
    assert [(i, m) for i, m, _ in pairs] == [(3, 1), (2, 0)] and sm == [2] and ss == []
    # without bundling saddles 10 and 11 also join 0 and 1 (costs 3 and 2);
    # after 13's merge they and 12 join 0 and 2, 12 being the highest is
    # cancelled, and 10, 11 are left joining the single maximum 2: no cost,
    # so they stay in the graph with a one-entry row
    sm, ss, rows, pairs = S.cancel(maxima, mv, saddles, sv, offs, arcs, 10.0)
    assert [(i, m) for i, m, _ in pairs] == [(3, 1), (2, 0)]
    assert sm == [2] and ss == [0, 1] and rows == [[2], [2]]


def test_multi_saddle_cost_is_gap_to_second_highest_maximum():
    # one saddle at height 1 joins maxima of heights 10, 9 and 2.  Its cost is
    # 9 - 1 = 8 (the second-highest maximum), not 2 - 1 = 1 (the lowest)
    g = _hand([10.0, 9.0, 2.0], [1.0], [[0, 1, 2]])
    for t in (5.0, 7.999):
        sm, ss, rows, pairs = S.cancel(*g, t)
        assert pairs == [] and sm == [0, 1, 2] and ss == [0] and rows == [[0, 1, 2]]
    # at cost <= threshold one cancellation removes the saddle and merges
    # both lower maxima into the highest (the surviving maximum)
    for t in (8.0, 100.0):
        sm, ss, rows, pairs = S.cancel(*g, t)
        assert pairs == [(0, 1, 8.0), (0, 2, 8.0)]
        assert sm == [0] and ss == [] and rows == []
    # the minimum graph of the negated values is the same graph
    gm = (g[0], -g[1], g[2], -g[3], g[4], g[5])
    assert S.cancel(*gm, 100.0, minima=True)[3] == [(0, 1, 8.0), (0, 2, 8.0)]


def test_multi_saddle_order_differs_from_elder_rule():
    # saddle A (height 1) joins maxima 10, 9, 2; saddle B (height 0.5) joins
    # maxima 2 and 3.  Costs: A = 9 - 1 = 8, B = 2 - 0.5 = 1.5.  B goes first
    # and merges 2 into 3; A then joins 10, 9, 3 and merges 9 and 3 into 10.
    # (The elder rule of superlevel sets would pair 2 with A at persistence 1
    # and 3 with B at persistence 2.5 instead.)
    g = _hand([10.0, 9.0, 2.0, 3.0], [1.0, 0.5], [[0, 1, 2], [2, 3]])
    sm, ss, rows, pairs = S.cancel(*g, np.inf)
    assert pairs == [(1, 2, 1.5), (0, 1, 8.0), (0, 3, 8.0)]
    assert sm == [0] and ss == []
    # threshold 5: B is cancelled; A then costs 8 and is discarded
    sm, ss, rows, pairs = S.cancel(*g, 5.0)
    assert pairs == [(1, 2, 1.5)] and sm == [0, 1, 3] and ss == [0] and rows == [[0, 1, 3]]


def test_reinsert_when_cost_grew():
    # saddle A (height 4) joins maxima 6 and 5 (cost 1); saddle B (height 4.5)
    # joins 5 and 20 (cost 0.5); C (height 3.2) joins 6 and 7 (cost 2.8).  B
    # goes first and merges 5 into 20; A now joins 6 and 20 and costs 2, still
    # below C's 2.8, so A is cancelled next (6 into 20); C then joins 7 and 20
    # and costs 7 - 3.2 = 3.8.
    g = _hand([6.0, 5.0, 20.0, 7.0], [4.0, 4.5, 3.2], [[0, 1], [1, 2], [0, 3]])
    sm, ss, rows, pairs = S.cancel(*g, np.inf)
    assert [(i, m) for i, m, _ in pairs] == [(1, 1), (0, 0), (2, 3)]
    assert [c for _, _, c in pairs] == pytest.approx([0.5, 2.0, 3.8])
    # now C sits at height 4.5 (cost 6 - 4.5 = 1.5) and B at 4.9 (cost 0.1).
    # B merges 5 into 20; A's recomputed cost 2 exceeds the cost stored at the
    # top of the queue (C, 1.5), so A is reinserted; C merges 6 into 7; A then
    # joins 7 and 20 and costs 7 - 4 = 3.  Cancelling A at cost 2 instead would
    # have merged 6 into 20.
    g = _hand([6.0, 5.0, 20.0, 7.0], [4.0, 4.9, 4.5], [[0, 1], [1, 2], [0, 3]])
    sm, ss, rows, pairs = S.cancel(*g, np.inf)
    assert [(i, m) for i, m, _ in pairs] == [(1, 1), (2, 0), (0, 3)]
    assert [c for _, _, c in pairs] == pytest.approx([0.1, 1.5, 3.0])
    assert sm == [2] and ss == []


def test_bundling_keeps_unshared_saddles():
    # saddle 0 joins only maximum 0 (both arcs to one maximum): no pair shares
    # it, so bundling keeps it; saddles 1 and 2 share the pair (0, 1), the
    # higher (2) represents it
    g = _hand([5.0, 4.0], [1.0, 2.0, 3.0], [[0], [0, 1], [0, 1]])
    assert S.bundle(*g) == [0, 2]


def test_1d_chain_bundling_keeps_everything():
    f = W.random_field((60,), 3, "uniform")
    g = _graph(f, False)
    kept = S.bundle(*g)
    # in 1D every saddle joins two different neighbours: no pair is shared
    assert kept == list(range(len(g[2])))


def _sines(shape, seed):
    """Sum of one sine per axis plus a slight tilt: a separable Morse-like
    field whose PL saddles all join at most two maxima."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = np.meshgrid(*[np.linspace(0, 1, d) for d in shape], indexing="ij")
    f = np.zeros(shape)
    for g in grids:
        f += np.sin(rng.uniform(4, 9) * g + rng.uniform(0, 2 * np.pi))
    f += sum(rng.uniform(0.01, 0.05) * g for g in grids)
    return f.astype(np.float32)


SIMPLE_FIELDS = [("uniform1d", (40,), 5), ("uniform1d", (60,), 8), ("mix", (30, 40), 5), ("mix", (24, 20), 2),
                 ("sines", (30, 40), 10), ("sines", (20, 18, 16), 10), ("sines", (9, 8, 7, 6), 4),
                 ("sines", (12, 11, 10, 9), 6)]


@pytest.mark.parametrize("kind,shape,seed", SIMPLE_FIELDS)
def test_cancellation_pairs_equal_elder_rule_on_simple_saddles(kind, shape, seed):
    if kind == "uniform1d":
        f = W.random_field(shape, seed, "uniform")
    elif kind == "mix":
        f = W.gaussian_mixture(shape, seed, n_gauss=5, noise=1e-3)
    else:
        f = _sines(shape, seed)
    for minima in (False, True):
        g = _graph(f, minima)
        offs, arcs = g[4], g[5]
        # precondition of the pin: every saddle joins at most two maxima, so
        # the second-highest maximum is the lowest and a cancellation merges
        # one maximum, as the elder rule does
        assert all(len(set(arcs[offs[i]:offs[i + 1]].tolist())) <= 2 for i in range(len(g[2])))
        sm, ss, rows, pairs = S.cancel(*g, np.inf, minima)
        assert len(pairs) >= 1
        sad = g[2]
        got = sorted((int(sad[i]), int(m), round(float(c), 5)) for i, m, c in pairs)
        want = sorted((int(v), int(m), round(float(p), 5))
                      for v, m, p in S.superlevel_pairs(f, lambda v: O.neighbours(f.shape, v).tolist(), minima))
        assert got == want
        assert len(sm) == 1 and all(len(r) == 1 for r in rows)  # one component: one maximum remains
        # a finite threshold cancels exactly the pairs that cost no more
        t = float(np.median([c for _, _, c in pairs]))
        sm2, _, _, pairs2 = S.cancel(*g, t, minima)
        assert sorted((i, m) for i, m, _ in pairs2) == sorted((i, m) for i, m, c in pairs if c <= t)
        assert len(sm2) == len(g[0]) - len(pairs2)


@pytest.mark.parametrize("shape,kind", [((30, 40), "uniform"), ((40, 40), "ties"), ((14, 12, 10), "uniform"),
                                        ((8, 7, 6, 5), "uniform")])
def test_full_cancellation_keeps_highest_maximum_of_each_part(shape, kind):
    """With no threshold every saddle that joins two maxima is eventually
    cancelled, and merges always go into a saddle's highest maximum, so the
    survivors are exactly the highest maximum of each connected part of the
    graph (maxima joined through saddles), found here by a separate union-find
    over the input arcs.  These fields have multi-saddles."""
    f = W.random_field(shape, 7, kind)
    for minima in (False, True):
        g = _graph(f, minima)
        maxima, mv, sad, sv, offs, arcs = g
        multi = sum(len(set(arcs[offs[i]:offs[i + 1]].tolist())) >= 3 for i in range(len(sad)))
        assert multi > 0
        comp = {int(m): int(m) for m in maxima}

        def find(x):
            while comp[x] != x:
                x = comp[x]
            return x

        for i in range(len(sad)):
            row = [int(m) for m in arcs[offs[i]:offs[i + 1]]]
            for m in row[1:]:
                a, b = find(row[0]), find(m)
                if a != b:
                    comp[a] = b
        h = dict(zip((int(m) for m in maxima), (-v if minima else v for v in np.asarray(mv, np.float64))))
        best = {}
        for m in comp:
            r = find(m)
            key = (h[m], -m if minima else m)
            if r not in best or key > best[r][0]:
                best[r] = (key, m)
        sm, ss, rows, pairs = S.cancel(*g, np.inf, minima)
        assert sm == sorted(m for _, m in best.values())
        assert len(pairs) == len(maxima) - len(sm)
        assert all(len(r) == 1 for r in rows)
        # every row of one cancellation shares its saddle and cost, and the
        # cancellations come in non-decreasing cost only where no multi-saddle
        # lowered a cost: at least the costs are all finite and >= 0
        assert all(np.isfinite(c) and c >= 0 for _, _, c in pairs)


def test_bundling_keeps_pair_connectivity():
    f = W.gaussian_mixture((48, 40), 9, n_gauss=6, noise=1e-3)
    maxima, mv, sad, sv, offs, arcs = _graph(f, False)
    kept = set(S.bundle(maxima, mv, sad, sv, offs, arcs))
    pairs_in, pairs_kept = set(), set()
    for i in range(len(sad)):
        ms = sorted(set(arcs[offs[i]:offs[i + 1]].tolist()))
        ps = {(a, b) for a in ms for b in ms if a < b}
        pairs_in |= ps
        if i in kept:
            pairs_kept |= ps
    assert pairs_in == pairs_kept and len(kept) < len(sad)


SIMPLIFY_MUTANTS = {
    # the cost of a multi-saddle taken against its lowest maximum
    "cost_lowest_maximum": ("return (hm[ms[1]] - hs[i], order_key(i), i)", "return (hm[ms[-1]] - hs[i], order_key(i), i)"),
    # a cancellation merges only the lowest maximum
    "merge_lowest_only": ("for m in ms[1:]:", "for m in ms[-1:]:"),
    # a saddle whose recomputed cost grew is cancelled anyway
    "no_reinsert": ("if heap and cost > heap[0][0]:", "if False:"),
    # merges go into the lowest maximum instead of the highest
    "lowest_survives": ("for m in ms[1:]:\n            parent[m] = ms[0]",
                        "for m in ms[:-1]:\n            parent[m] = ms[-1]"),
    # bundling drops saddles that no pair shares
    "bundle_drops_unshared": ("unshared.append(i)", "pass"),
}


@pytest.mark.parametrize("name", sorted(SIMPLIFY_MUTANTS))
def test_pins_catch_simplify_mutants(name, monkeypatch):
    """Each mutant is a copy of the reference with one plausible mistake
    planted in its source; at least one pin above must fail on it."""
    import types

    old, new = SIMPLIFY_MUTANTS[name]
    src = open(S.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("simplify_mutant")
    exec(compile(src.replace(old, new), S.__file__, "exec"), mod.__dict__)
    monkeypatch.setattr(__import__(__name__), "S", mod, raising=False)
    monkeypatch.setitem(globals(), "S", mod)
    pins = [test_hand_worked_bundling_and_cancellation, test_multi_saddle_cost_is_gap_to_second_highest_maximum,
            test_multi_saddle_order_differs_from_elder_rule, test_reinsert_when_cost_grew,
            test_bundling_keeps_unshared_saddles]
    failed = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, f"no pin catches the mutant {name}"
