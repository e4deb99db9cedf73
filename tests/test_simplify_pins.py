"""Pins of the simplification reference (oracle/simplify.py): a hand-worked
graph, the 1D chain, and persistence pairs equal to the textbook elder-rule
pairing of the superlevel sets, computed by union-find on the raw field."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import simplify as S
from paper_2303_02724_amd import workloads as W


def _graph(f, minima):
    g = O.extremum_graph(f, minima)
    fv = np.asarray(f, np.float32).reshape(-1)
    return (g["maxima"], fv[g["maxima"]], g["saddles"], fv[g["saddles"]], g["arc_offsets"], g["arc_maxima"])


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
    # first and merges maximum 1 into the elder 2; saddle 12 then joins 0 (5)
    # and 2 and costs 5 - 3 = 2 > 1: kept
    sm, ss, rows, pairs = S.cancel(maxima, mv, saddles, sv, offs, arcs, 1.0, keep=[2, 3])
    assert pairs == [(3, 1, 0.5)]
    assert sm == [0, 2] and ss == [2] and rows == [[0, 2]]
    # threshold 2: then saddle 12 merges maximum 0 into maximum 2
    sm, ss, rows, pairs = S.cancel(maxima, mv, saddles, sv, offs, arcs, 2.0, keep=[2, 3])
    assert [(i, m) for i, m, _ in pairs] == [(3, 1), (2, 0)] and sm == [2] and ss == []
    # without bundling saddles 10 and 11 also join 0 and 1 (costs 3 and 2);
    # after 13's merge they and 12 join 0 and 2, 12 being the highest is
    # cancelled, and 10, 11 are left joining a single maximum: dropped
    sm, ss, rows, pairs = S.cancel(maxima, mv, saddles, sv, offs, arcs, 10.0)
    assert [(i, m) for i, m, _ in pairs] == [(3, 1), (2, 0)] and ss == []


def test_1d_chain_bundling_keeps_everything():
    f = W.random_field((60,), 3, "uniform")
    g = _graph(f, False)
    kept = S.bundle(*g)
    # in 1D every saddle joins two different neighbours: no pair is shared
    assert kept == list(range(len(g[2])))


@pytest.mark.parametrize("shape,kind", [((40,), "uniform"), ((30, 40), "mix"), ((20, 18, 16), "mix"),
                                        ((12, 11, 10), "uniform"), ((9, 8, 7, 6), "uniform")])
def test_cancellation_pairs_equal_elder_rule(shape, kind):
    f = (W.gaussian_mixture(shape, 5, n_gauss=5, noise=1e-3) if kind == "mix"
         else W.random_field(shape, 5, kind))
    for minima in (False, True):
        g = _graph(f, minima)
        sm, ss, rows, pairs = S.cancel(*g, np.inf, minima)
        sad = g[2]
        got = sorted((int(sad[i]), int(m), round(float(c), 5)) for i, m, c in pairs)
        want = sorted((int(v), int(m), round(float(p), 5))
                      for v, m, p in S.superlevel_pairs(f, lambda v: O.neighbours(f.shape, v).tolist(), minima))
        assert got == want
        assert len(sm) == 1 and ss == []  # one component: one maximum remains
        # a finite threshold cancels exactly the pairs that cost no more
        t = float(np.median([c for _, _, c in pairs]))
        sm2, _, _, pairs2 = S.cancel(*g, t, minima)
        assert sorted((i, m) for i, m, _ in pairs2) == sorted((i, m) for i, m, c in pairs if c <= t)
        assert len(sm2) == len(g[0]) - len(pairs2)


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
