"""Plain reference for extremum-graph simplification (the paper's Sec. 3.5:
arc bundling and persistence-directed cancellation).

TEST INFRASTRUCTURE ONLY.  Only the tests may use it; the library never does.
Written for clarity: dictionaries, sets and a binary heap, following the
steps in the order Sec. 3.5 gives them.

Readings (the paper describes the operations in prose; these are the
choices written out):

* Order.  Critical points compare by value, ties by vertex id (the
  simulated perturbation of Sec. 3.3); for the minimum graph the order is
  reversed.  ``height(v)`` below is the value in the graph's own direction
  (f for the maximum graph, -f for the minimum graph).
* Arc bundling.  For every pair of maxima that share a saddle, the highest
  shared saddle represents the pair and the other saddles the pair shares
  are discarded.  A saddle is kept iff it represents at least one pair of its
  maxima (so every connected pair stays connected), or iff it has fewer than
  two distinct maxima (then no pair shares it and nothing discards it).
* Persistence-directed cancellation, threshold t.  The maxima of a saddle
  are the representatives (after earlier merges) of its arcs' maxima.  The
  cost of a saddle is height(second-highest of its maxima) - height(saddle):
  for a simple saddle (two maxima) this is the smaller gap to its two
  maxima, for a multi-saddle the gap to the second-highest maximum.  A saddle
  with fewer than two distinct maxima has no cost and cannot be cancelled.
  The queue starts with every saddle that has a cost, ordered by (cost, then
  the saddle's order: lower first).  The top is popped and its cost
  recomputed: no cost -> dropped; cost > t -> discarded; cost greater than
  the cost stored at the new top of the queue -> reinserted; otherwise the
  saddle is cancelled: every one of its maxima except the highest (the
  surviving maximum) merges into the highest, and the saddle leaves the graph.
  A cancellation is reported as one row (saddle, merged maximum, cost) per
  merged maximum, the merged maxima from the highest down.
* Output.  Surviving maxima are those never merged; surviving saddles are the
  kept saddles that were not cancelled, each with the sorted distinct
  representatives of its arcs' maxima as its arc row (a single entry when
  all its maxima merged into one).
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
    unshared = []
    for i in range(len(saddles)):
        ms = sorted(set(int(x) for x in arc_maxima[arc_offsets[i]:arc_offsets[i + 1]]))
        if len(ms) < 2:
            unshared.append(i)
        for a in range(len(ms)):
            for b in range(a + 1, len(ms)):
                k = (ms[a], ms[b])
                j = best.get(k)
                if j is None or _above(hs[i], int(saddles[i]), hs[j], int(saddles[j]), minima):
                    best[k] = i
    return sorted(set(best.values()) | set(unshared))


def cancel(maxima, max_values, saddles, sad_values, arc_offsets, arc_maxima, threshold, minima=False,
           keep=None):
    """Persistence-directed cancellation.  ``keep`` optionally restricts the
    input to those saddle indices (e.g. the survivors of bundling).

    Returns (surviving maxima, surviving saddle indices, their arc rows,
    cancellation rows (saddle index, merged maximum, cost) in order).
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

    def maxima_of(i):
        """Distinct current maxima of saddle i, highest first."""
        ms = list({find(m) for m in arcs[i]})
        ms.sort(key=lambda m: (hm[m], -m if minima else m), reverse=True)
        return ms

    def order_key(i):
        # the saddle's rank in the order, for ties in cost: lower saddles first
        s = int(saddles[i])
        return (hs[i], -s if minima else s)

    def entry(i):
        ms = maxima_of(i)
        if len(ms) < 2:
            return None
        return (hm[ms[1]] - hs[i], order_key(i), i)

    heap = [e for e in (entry(i) for i in arcs) if e is not None]
    heapq.heapify(heap)
    pairs = []
    cancelled = set()
    while heap:
        _, _, i = heapq.heappop(heap)
        e = entry(i)
        if e is None:
            continue
        cost = e[0]
        if cost > threshold:
            continue
        if heap and cost > heap[0][0]:
            heapq.heappush(heap, e)
            continue
        ms = maxima_of(i)
        for m in ms[1:]:
            parent[m] = ms[0]
            pairs.append((i, m, cost))
        cancelled.add(i)
    surv_max = sorted(m for m in parent if find(m) == m)
    surv_sad, rows = [], []
    for i in sorted(arcs):
        if i not in cancelled:
            surv_sad.append(i)
            rows.append(sorted({find(m) for m in arcs[i]}))
    return surv_max, surv_sad, rows, pairs


def superlevel_pairs(f, neighbours, minima=False):
    """Textbook 0-dimensional persistence of the superlevel sets (sublevel
    sets for the minimum graph) by union-find over the vertices in
    decreasing order, the elder rule deciding which component dies at a
    merge: a list of (vertex where a component dies, its maximum, persistence).
    ``neighbours(v)`` gives the grid neighbours of v.  Independent of the
    extremum graph; used to pin ``cancel`` on graphs whose saddles are all
    simple (there the cancellation order is the elder rule's)."""
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
