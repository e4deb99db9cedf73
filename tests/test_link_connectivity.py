"""The saddle test of the 4D-6D classification kernels decides whether an
upper link is connected by set algebra on the link's rows (eg_link.h).  Here
it is checked, on the host, against the definition: the link vertices are
the rows of Alg. 1 (the non-zero offsets in {0,1}^n or {0,-1}^n), two of
them joined iff their difference is again such an offset, and a mask is
connected iff a breadth-first search from one of its rows reaches all of
them; the component that the stage (d) kernels take apart is the one the
search reaches from the lowest row.  Masks: every mask for n <= 3, random masks of every density, and
the upper links of every interior vertex of random fields (n = 2..6)."""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def rows(n):
    """Alg. 1's offsets in lexicographic order (axis 0 first, -1 < 0 < 1)."""
    out = []
    for d in itertools.product((-1, 0, 1), repeat=n):
        if any(d) and (set(d) <= {0, 1} or set(d) <= {0, -1}):
            out.append(d)
    return np.array(out, dtype=np.int64)


def adjacency(n):
    r = rows(n)
    diff = r[:, None, :] - r[None, :, :]
    nz = diff.any(-1)
    return nz & (((diff >= 0) & (diff <= 1)).all(-1) | ((diff <= 0) & (diff >= -1)).all(-1))


def component(n, masks):
    """BFS from the lowest row of each mask, all masks at once: the rows
    reached."""
    A = adjacency(n).astype(np.float32)
    first = np.argmax(masks, axis=1)
    comp = np.zeros_like(masks)
    comp[np.arange(len(masks)), first] = True
    while True:
        grown = comp | (((comp.astype(np.float32) @ A) > 0) & masks)
        if np.array_equal(grown, comp):
            return comp
        comp = grown


def field_links(n, side, seed):
    """Upper-link masks of the interior vertices of a white-noise field."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((side,) * n)
    inner = tuple(slice(1, side - 1) for _ in range(n))
    c = f[inner]
    bits = []
    for d in rows(n):
        sl = tuple(slice(1 + di, side - 1 + di) for di in d)
        bits.append((f[sl] > c).reshape(-1))
    return np.stack(bits, 1)


def masks_for(n, rng):
    k = 2 * (2 ** n - 1)
    if k <= 14:
        ms = ((np.arange(1, 2 ** k)[:, None] >> np.arange(k)) & 1).astype(bool)
    else:
        p = rng.uniform(0.02, 0.98, size=(6000, 1))
        ms = rng.random((6000, k)) < p
    side = {2: 40, 3: 16, 4: 8, 5: 6, 6: 4}.get(n)
    if side:
        ms = np.concatenate([ms, field_links(n, side, 100 + n)])
    return ms[ms.any(1)]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("link") / "link_check")
    src = os.path.join(ROOT, "tests", "link_connected_check.cpp")
    inc = os.path.join(ROOT, "paper_2303_02724_amd", "csrc")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", inc, src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_link_connected_matches_bfs(checker, n):
    rng = np.random.default_rng(n)
    ms = masks_for(n, rng)
    comp = component(n, ms)
    want = (comp == ms).all(1)
    bits = 1 << np.arange(ms.shape[1], dtype=object)
    w = (ms.astype(object) * bits).sum(1)
    wc = (comp.astype(object) * bits).sum(1)
    lines = "".join(f"{n} {int(x) >> 64:x} {int(x) & ((1 << 64) - 1):x}\n" for x in w)
    r = subprocess.run([checker], input=lines, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = r.stdout.split()
    got = np.array([c == "1" for c in out[0::3]])
    got_comp = np.array([(int(h, 16) << 64) | int(l, 16) for h, l in zip(out[1::3], out[2::3])], dtype=object)
    assert got.shape == want.shape and got_comp.shape == wc.shape
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"n={n}: connectivity of {bad.size} of {len(ms)} masks differs, first {w[bad[0]]:#x}"
    bad = np.flatnonzero(got_comp != wc)
    assert bad.size == 0, f"n={n}: component of {bad.size} of {len(ms)} masks differs, first {w[bad[0]]:#x}"
    # both kinds occur (except n = 1, where a single row is always connected)
    if n >= 2:
        assert want.any() and (~want).any()
