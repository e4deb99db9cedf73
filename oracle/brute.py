"""Literal brute-force extremum graph for tiny grids (pure Python).

TEST INFRASTRUCTURE ONLY.  It pins the C oracle: everything is done the
slowest, most literal way, straight from the paper's definitions.

* Edges: GridAdjacency (Alg. 1) evaluated on *every pair* of grid vertices.
* Order: simulated perturbation, compared as Python tuples (f[v], v); the
  minimum graph compares (-f[v], -v), i.e. the reversed order.  Integer and
  float64 samples become Python ints and floats, which compare exactly;
  other types are converted to float32 first.
* Link, upper link, beta+: Sec. 3.3 and Table 1; components by BFS over the
  upper link with the link edges taken from the global edge set.
* Gradient: the highest vertex of the upper link (Sec. 3.3).
* Paths: Alg. 2 as written -- for each rep of a saddle (UpperLinkRep, the
  highest vertex of each upper-link component) follow the gradient until a
  maximum is reached; the arc is (saddle, that maximum).
* Labels: the same walk started at every vertex.
"""
from __future__ import annotations

import itertools
from collections import deque

import numpy as np


def grid_adjacency(p, q) -> bool:
    """Alg. 1: the set of coordinate differences lies in {0,1} or in {0,-1}."""
    U = set()
    for i in range(len(p)):
        U.add(p[i] - q[i])
    return p != q and (U <= {0, 1} or U <= {0, -1})


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

    # all-pairs edge set
    adj = [[] for _ in range(N)]
    for a in range(N):
        for b in range(a + 1, N):
            if grid_adjacency(verts[a], verts[b]):
                adj[a].append(b)
                adj[b].append(a)
    adjset = [set(x) for x in adj]

    beta = [0] * N
    grad = list(range(N))
    reps_of = {}
    for v in range(N):
        upper = [u for u in adj[v] if key(u) > key(v)]
        if upper:
            grad[v] = max(upper, key=key)
        seen = set()
        comps = []
        for u in upper:
            if u in seen:
                continue
            comp = []
            dq = deque([u])
            seen.add(u)
            while dq:
                x = dq.popleft()
                comp.append(x)
                for y in upper:
                    if y not in seen and y in adjset[x]:
                        seen.add(y)
                        dq.append(y)
            comps.append(comp)
        beta[v] = len(comps)
        reps_of[v] = [max(c, key=key) for c in comps]

    M = {v for v in range(N) if beta[v] == 0}

    labels = []
    for v in range(N):
        u = v
        while u not in M:
            u = grad[u]
        labels.append(u)

    saddles = [v for v in range(N) if beta[v] >= 2]
    rows = []
    paths = {}
    for s in saddles:
        P = []
        for u in reps_of[s]:
            p = [s]
            while u not in M:
                p.append(u)
                u = grad[u]
            P.append((p, u))
        paths[s] = P
        rows.append(sorted({u for (_, u) in P}))

    offsets = [0]
    for r in rows:
        offsets.append(offsets[-1] + len(r))
    return {
        "ptr": np.array(grad, dtype=np.int32),
        "beta": np.array(beta, dtype=np.int32),
        "labels": np.array(labels, dtype=np.int32),
        "maxima": np.array(sorted(M), dtype=np.int32),
        "saddles": np.array(saddles, dtype=np.int32),
        "saddle_beta": np.array([beta[s] for s in saddles], dtype=np.int32),
        "arc_offsets": np.array(offsets, dtype=np.int32),
        "arc_maxima": np.array([m for r in rows for m in r], dtype=np.int32),
        "reps": {s: sorted(reps_of[s]) for s in saddles},
        "paths": paths,
        "degree": [len(a) for a in adj],
        "adj": adj,
    }
