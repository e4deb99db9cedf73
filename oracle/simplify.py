"""Plain reference for extremum-graph simplification (the paper's Sec. 3.5:
arc bundling and persistence-directed cancellation).

TEST INFRASTRUCTURE ONLY.  Only the tests may use it; the library never does.
Written for clarity: dictionaries, sets and a binary heap, following the
steps as the paper describes them.

Readings (the paper describes the operations in prose; these are the
choices written out):

* Order.  Critical points compare by value, ties by vertex id (the
  simulated perturbation of Sec. 3.3); for the minimum graph the order is
  reversed.  ``height(v)`` below is the value in the graph's own direction
  (f for the maximum graph, -f for the minimum graph).
* Arc bundling.  For every pair of maxima that share a saddle, the highest
  shared saddle represents the pair.  A saddle survives iff it represents at
  least one pair of its maxima, so every connected pair stays connected.
  Saddles with fewer than two maxima have no pair and are dropped.
* Persistence-directed cancellation, threshold t.  A saddle's maxima are
  the representatives (after earlier merges) of its arcs' maxima; a saddle
  with fewer than two distinct ones is not a candidate.  cost(s) =
  height(lowest maximum) - height(s).  Saddles sit in a priority queue
  ordered by (cost, then the saddle's order); the top is popped, its cost
  recomputed: not a candidate -> dropped; cost > t -> discarded (costs never
  fall); cost above the new top's -> reinserted; otherwise cancelled: the
  lowest maximum m merges into the highest maximum of the saddle (the elder)
  and the pair (s, m) is recorded.  A saddle with more maxima left after the
  merge goes back into the queue, so a k-fold saddle can be cancelled k-1
  times.  At the end, surviving maxima are those never merged; surviving
  saddles those with at least two distinct maxima, whose arcs are those
  maxima.
"""
from __future__ import annotations

import heapq

import numpy as np


def _heights(values, minima):
    v = np.asarray(values, dtype=np.float64)
    return -v if minima else v


def _above(ha, ia, hb, ib, minima):
    """a above b in the graph's order: height, then vertex id (reversed for
    the minimum graph)."""
    if ha != hb:
        return ha > hb
    return ia < ib if minima else ia > ib


def bundle(maxima, max_values, saddles, sad_values, arc_offsets, arc_maxima, minima=False):
    """Indices (into ``saddles``) of the saddles that survive arc bundling."""
    hs = _heights(sad_values, minima)
    best = {}  # (ma, mb) -> saddle index
    for i in range(len(saddles)):
        ms = sorted(set(int(x) for x in arc_maxima[arc_offsets[i]:arc_offsets[i + 1]]))
        for a in range(len(ms)):
            for b in range(a + 1, len(ms)):
                k = (ms[a], ms[b])
                j = best.get(k)
                if j is None or _above(hs[i], int(saddles[i]), hs[j], int(saddles[j]), minima):
                    best[k] = i
    return sorted(set(best.values()))


def cancel(maxima, max_values, saddles, sad_values, arc_offsets, arc_maxima, threshold, minima=False,
           keep=None):
    """Persistence-directed cancellation.  ``keep`` optionally restricts the
    input to those saddle indices (e.g. the survivors of bundling).

    Returns (surviving maxima, surviving saddle indices, their arc rows,
    cancelled pairs as (saddle index, maximum, cost) in cancellation order).
    """
    hm = dict(zip((int(m) for m in maxima), _heights(max_values, minima)))
    hs = _heights(sad_values, minima)
    idx = range(len(saddles)) if keep is None else keep
    arcs = {i: set(int(x) for x in arc_maxima[arc_offsets[i]:arc_offsets[i + 1]]) for i in idx}
    parent = {int(m): int(m) for m in maxima}

    def find(m):
        while parent[m] != m:
            parent[m] = parent[parent[m]]
            m = parent[m]
        return m

    def lowest_highest(i):
        ms = sorted({find(m) for m in arcs[i]})
        lo = hi = None
        for m in ms:
            if lo is None or _above(hm[lo], lo, hm[m], m, minima):
                lo = m
            if hi is None or _above(hm[m], m, hm[hi], hi, minima):
                hi = m
        return len(ms), lo, hi

    def order_key(i):
        # the saddle's rank in the order, for ties in cost: lower saddles first
        s = int(saddles[i])
        return (hs[i], -s if minima else s)

    def entry(i):
        n, lo, _ = lowest_highest(i)
        if n < 2:
            return None
        return (hm[lo] - hs[i], order_key(i), i)

    heap = [e for e in (entry(i) for i in arcs) if e is not None]
    heapq.heapify(heap)
    pairs = []
    while heap:
        _, _, i = heapq.heappop(heap)
        e = entry(i)
        if e is None:
            continue
        if e[0] > threshold:
            continue
        if heap and e[:2] > heap[0][:2]:
            heapq.heappush(heap, e)
            continue
        _, lo, hi = lowest_highest(i)
        parent[lo] = hi
        pairs.append((i, lo, e[0]))
        e2 = entry(i)
        if e2 is not None:
            heapq.heappush(heap, e2)
    surv_max = sorted(m for m in parent if find(m) == m)
    surv_sad, rows = [], []
    for i in sorted(arcs):
        ms = sorted({find(m) for m in arcs[i]})
        if len(ms) >= 2:
            surv_sad.append(i)
            rows.append(ms)
    return surv_max, surv_sad, rows, pairs


def superlevel_pairs(f, neighbours, minima=False):
    """Textbook 0-dimensional persistence of the superlevel sets (sublevel
    sets for the minimum graph) by union-find over the vertices in
    decreasing order, the elder rule deciding which component dies at a
    merge: a list of (vertex where a component dies, its maximum, persistence).
    ``neighbours(v)`` gives the grid neighbours of v.  Independent of the
    extremum graph; used to pin ``cancel``."""
    vals = np.asarray(f, dtype=np.float64).reshape(-1)
    h = -vals if minima else vals
    n = vals.size
    order = sorted(range(n), key=lambda v: (h[v], -v if minima else v), reverse=True)
    parent = {}
    top = {}  # component root -> its maximum

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    pairs = []
    for v in order:
        parent[v] = v
        top[v] = v
        roots = {find(u) for u in neighbours(v) if u in parent and u != v}
        if not roots:
            continue
        # the elder (highest maximum) absorbs the others, which die here
        rs = sorted(roots, key=lambda r: (h[top[r]], -top[r] if minima else top[r]), reverse=True)
        elder = rs[0]
        for r in rs[1:]:
            pairs.append((v, top[r], h[top[r]] - h[v]))
            parent[r] = elder
        parent[v] = elder
    return pairs
