"""eg_build_noalloc (the entry point that allocates nothing: its workspace is
the library's fixed per-device scratch array) against eg_build through the C
ABI, bit-exact, on consecutive calls that reuse the same scratch: a 3D field,
then a smaller 2D field, then a smaller 3D field in the minimum graph."""
import numpy as np
import pytest
import torch

from paper_2303_02724_amd import eg, workloads as W

pytestmark = pytest.mark.gpu

KEYS = ["labels", "maxima", "saddles", "saddle_beta", "arc_offsets", "arc_maxima", "ptr"]


def _host(r):
    return {
        "labels": r.labels.reshape(-1).cpu().numpy(),
        "maxima": r.maxima.cpu().numpy(),
        "saddles": r.saddles.cpu().numpy(),
        "saddle_beta": r.saddle_beta.cpu().numpy(),
        "arc_offsets": r.arc_offsets.cpu().numpy(),
        "arc_maxima": r.arc_maxima.cpu().numpy(),
        "ptr": r.ptr.reshape(-1).cpu().numpy(),
    }


def _both(f: np.ndarray, minima: bool):
    t = torch.from_numpy(f).to("cuda:0")
    ref = eg.Builder(f.shape, minima=minima, want_ptr=True, device=t.device)
    na = eg.Builder(f.shape, minima=minima, want_ptr=True, device=t.device, noalloc=True)
    assert na.ws is None and na.out.workspace is None
    a = _host(ref.run(t))
    b = _host(na.run(t))
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (f.shape, minima, k)
    return a


def test_noalloc_equals_build_on_consecutive_calls():
    cases = [
        (W.gaussian_random_field((70, 96, 130), 11, corr_len=3.0, workers=4), False),  # 873,600 vertices, many tiles
        (W.gaussian_mixture((300, 257), 12, n_gauss=8, noise=1e-3), False),            # smaller, 2D, ragged tiles
        (W.gaussian_random_field((30, 40, 60), 13, corr_len=2.0, workers=4), True),     # smaller again, minimum graph
    ]
    sizes = [f.size for f, _ in cases]
    assert sizes == sorted(sizes, reverse=True)
    for f, minima in cases:
        print(f"noalloc case {f.shape} minima={minima}", flush=True)
        a = _both(f, minima)
        assert a["maxima"].size > 0 and a["saddles"].size > 0
