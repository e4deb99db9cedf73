"""GPU parity of the streamed build (eg_build_streamed): a host-resident field
copied slab by slab along the slowest axis while the slabs that have landed
are classified gives exactly the oracle's graph, for slab sizes that are a
single tile row, several, not a multiple of the tile depth, and the whole
field, in both graphs, 2D and 3D."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2303_02724_amd import eg, workloads as W
from tests.gpu_util import KEYS, assert_same

pytestmark = pytest.mark.gpu


def _pinned(f):
    t = torch.empty(f.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(f)))
    return t


def _np(r):
    out = {"labels": r.labels.reshape(-1).cpu().numpy(), "maxima": r.maxima.cpu().numpy(),
           "saddles": r.saddles.cpu().numpy(), "saddle_beta": r.saddle_beta.cpu().numpy(),
           "arc_offsets": r.arc_offsets.cpu().numpy(), "arc_maxima": r.arc_maxima.cpu().numpy()}
    if r.ptr is not None:
        out["ptr"] = r.ptr.reshape(-1).cpu().numpy()
    return out


@pytest.mark.parametrize("slab", [1, 8, 13, 70])
def test_streamed_3d_equals_oracle(slab):
    f = W.gaussian_random_field((70, 96, 130), 31, corr_len=3.0, workers=4)
    host = _pinned(f)
    for minima in (False, True):
        print(f"streamed 3d slab={slab} minima={minima}", flush=True)
        r = eg.build_streamed(host, slab, minima=minima, want_ptr=True)
        assert_same(_np(r), O.extremum_graph(f, minima), KEYS + ["ptr"], f"streamed slab={slab} minima={minima}")


@pytest.mark.parametrize("tile3", [1, 2])
def test_streamed_3d_other_tiles(tile3):
    f = W.gaussian_random_field((45, 40, 70), 32, corr_len=2.0, workers=4)
    r = eg.build_streamed(_pinned(f), 9, want_ptr=True, tuning=eg.tuning(tile3=tile3))
    assert_same(_np(r), O.extremum_graph(f), KEYS + ["ptr"], f"streamed tile3={tile3}")


@pytest.mark.parametrize("slab", [1, 5, 40])
def test_streamed_2d_equals_oracle(slab):
    f = W.gaussian_mixture((300, 257), 33, n_gauss=8, noise=1e-3)
    host = _pinned(f)
    for minima in (False, True):
        r = eg.build_streamed(host, slab, minima=minima, want_ptr=True)
        assert_same(_np(r), O.extremum_graph(f, minima), KEYS + ["ptr"], f"streamed 2d slab={slab}")


def test_streamed_rejects_bad_arguments():
    f = W.gaussian_mixture((64, 64), 34)
    b = eg.Builder(f.shape)
    with pytest.raises(eg.EGError):
        b.launch_streamed(torch.from_numpy(f).cuda(), 8)  # must be host memory
    with pytest.raises(eg.EGError):
        b.launch_streamed(_pinned(f), 0)  # slab_planes < 1
    b5 = eg.Builder((4, 4, 4, 4))
    with pytest.raises(eg.EGError):
        b5.launch_streamed(_pinned(np.zeros((4, 4, 4, 4), np.float32)), 2)  # 4D is not streamed
