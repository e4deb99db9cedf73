"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
bring the results back as numpy arrays shaped like the oracle's."""
import numpy as np
import torch

from paper_2303_02724_amd import eg

KEYS = ["labels", "maxima", "saddles", "saddle_beta", "arc_offsets", "arc_maxima"]


def gpu_graph(f: np.ndarray, minima: bool = False, want_ptr: bool = True, tuning: int = 0, **caps) -> dict:
    t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to("cuda:0")
    r = eg.build(t, minima=minima, want_ptr=want_ptr, tuning=tuning, **caps)
    out = {
        "labels": r.labels.reshape(-1).cpu().numpy(),
        "maxima": r.maxima.cpu().numpy(),
        "saddles": r.saddles.cpu().numpy(),
        "saddle_beta": r.saddle_beta.cpu().numpy(),
        "arc_offsets": r.arc_offsets.cpu().numpy(),
        "arc_maxima": r.arc_maxima.cpu().numpy(),
        "passes": r.passes,
    }
    if r.ptr is not None:
        out["ptr"] = r.ptr.reshape(-1).cpu().numpy()
    return out


def assert_same(gpu: dict, ora: dict, keys=KEYS, ctx=""):
    for k in keys:
        a, b = np.asarray(gpu[k]), np.asarray(ora[k])
        if not np.array_equal(a, b):
            if a.shape != b.shape:
                raise AssertionError(f"{ctx} {k}: shape {a.shape} vs oracle {b.shape}")
            bad = np.flatnonzero(a != b)
            raise AssertionError(f"{ctx} {k}: {bad.size} mismatches, first at {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
