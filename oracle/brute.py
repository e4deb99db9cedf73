"""Brute-force extremum graph for tiny grids (pure Python).

TEST INFRASTRUCTURE ONLY.  It pins the C oracle: everything is computed the
slowest way, from the definitions, in a different form from the oracle's.

* Edges (Alg. 1): the Freudenthal tessellation puts two distinct grid points
  in a common simplex iff they are comparable in the component-wise order and
  at Chebyshev distance 1.  This is tested on *every pair* of grid vertices.
* Order: simulated perturbation (Sec. 3.3), compared as Python tuples
  (f[v], v); the minimum graph compares (-f[v], -v), i.e. the reversed order.
  Integer and float64 samples become Python ints and floats, which compare
  exactly; other types are converted to float32 first.
* Link, upper link, beta+: Sec. 3.3 and Table 1; components by breadth-first
  search over the upper link, edges taken from the global edge set,
  components listed by their smallest vertex id.
* Gradient: the highest vertex of the upper link (Sec. 3.3); a maximum is its
  own target.
* Labels and paths (Sec. 2, Alg. 2): the vertices are visited from the highest
  down, so a vertex's gradient target has always been visited before it: a
  maximum is its own label and its path is itself; any other vertex takes its
  target's label, and its path is itself followed by its target's path.  For a
  saddle s, the path of the highest vertex r of each upper-link component
  (UpperLinkRep) prefixed by s is the gradient path from s through that
  component, and its last vertex is the arc's maximum.
"""
from __future__ import annotations

import itertools
from collections import deque

import numpy as np


def grid_adjacency(p, q) -> bool:
    """Alg. 1: p and q span an edge of the Freudenthal tessellation: they
    differ, one dominates the other coordinate-wise, and no coordinate differs
    by more than one."""
    d = [b - a for a, b in zip(p, q)]
    if not any(d) or max(abs(x) for x in d) > 1:
        return False
    return all(x >= 0 for x in d) or all(x <= 0 for x in d)


def extremum_graph(f, minima: bool = False) -> dict:
    f = np.asarray(f)
    if not (np.issubdtype(f.dtype, np.integer) or f.dtype in (np.float32, np.float64)):
        f = f.astype(np.float32)
    shape = f.shape
    verts = list(itertools.product(*[range(d) for d in shape]))  # C order
    N = len(verts)
    vals = f.reshape(-1).tolist()

    def key(v):
        return (-vals[v], -v) if minima else (vals[v], v)

    # all-pairs edge set; neighbour lists come out ascending
    nbrs = [[] for _ in range(N)]
    for a, b in itertools.combinations(range(N), 2):
        if grid_adjacency(verts[a], verts[b]):
            nbrs[a].append(b)
            nbrs[b].append(a)
    for lst in nbrs:
        lst.sort()
    nbr_sets = [set(x) for x in nbrs]

    beta = [0] * N
    target = list(range(N))
    reps_of = {}
    for v in range(N):
        upper = [u for u in nbrs[v] if key(u) > key(v)]
        if upper:
            target[v] = max(upper, key=key)
        comp_of = {}
        comps = []
        for u in upper:  # ascending: a component is found at its smallest vertex
            if u in comp_of:
                continue
            comp_of[u] = len(comps)
            members = [u]
            frontier = deque([u])
            while frontier:
                x = frontier.popleft()
                for y in upper:
                    if y not in comp_of and y in nbr_sets[x]:
                        comp_of[y] = len(comps)
                        members.append(y)
                        frontier.append(y)
            comps.append(members)
        beta[v] = len(comps)
        reps_of[v] = [max(c, key=key) for c in comps]

    # labels and gradient paths, highest vertex first
    label = [None] * N
    path = [None] * N
    for v in sorted(range(N), key=key, reverse=True):
        if beta[v] == 0:
            label[v], path[v] = v, (v,)
        else:
            t = target[v]
            label[v], path[v] = label[t], (v,) + path[t]

    maxima = [v for v in range(N) if beta[v] == 0]
    saddles = [v for v in range(N) if beta[v] >= 2]
    paths = {s: [[s] + list(path[r]) for r in reps_of[s]] for s in saddles}
    rows = [sorted({p[-1] for p in paths[s]}) for s in saddles]

    offsets = [0]
    for r in rows:
        offsets.append(offsets[-1] + len(r))
    return {
        "ptr": np.array(target, dtype=np.int32),
        "beta": np.array(beta, dtype=np.int32),
        "labels": np.array(label, dtype=np.int32),
        "maxima": np.array(maxima, dtype=np.int32),
        "saddles": np.array(saddles, dtype=np.int32),
        "saddle_beta": np.array([beta[s] for s in saddles], dtype=np.int32),
        "arc_offsets": np.array(offsets, dtype=np.int32),
        "arc_maxima": np.array([m for r in rows for m in r], dtype=np.int32),
        "reps": {s: sorted(reps_of[s]) for s in saddles},
        "paths": paths,
        "degree": [len(a) for a in nbrs],
        "adj": nbrs,
    }
