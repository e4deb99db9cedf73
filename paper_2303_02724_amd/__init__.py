"""MI355X-native extremum graphs of piecewise-linear scalar fields on grids.

The HIP library (``csrc/``, built into ``libeg_hip.so``) computes, for a
float32 field on an n-D grid (n = 1..6) with the Freudenthal tessellation:
steepest-ascent pointers, per-vertex labels (the maximum of each vertex's
descending manifold), maxima, (n-1)-saddles with their upper-link component
counts, and the de-duplicated saddle-maximum arcs in CSR form.

``paper_2303_02724_amd.eg`` is the thin Python binding (argument marshalling
only).  It is imported lazily so that ``workloads`` can be used without the
HIP runtime.
"""

__all__ = ["eg", "workloads"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
