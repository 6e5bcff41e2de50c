"""raybornhf on MI355X: one Hessian-free ray-Born frequency step (arXiv 2211.00316) as
hand-written HIP kernels for gfx950 behind a C ABI (include/raybornhf.h).

The Python side only marshals arguments; see paper_2211_00316_amd._lib.Context.
"""
from __future__ import annotations


__all__ = ["lib", "setup_for", "LIB_PATH"]


def lib():
    """The ctypes binding module (loads the shared library on first use)."""
    from . import _lib

    _lib.load()
    return _lib


def setup_for(w):
    """C-ABI structs (grid, ring, trace parameters) of a phantoms.Workload."""
    from . import _lib

    grid = _lib.Grid(w.nx, w.ny, w.dx, w.x0, w.y0, w.mask_radius)
    ring = _lib.Ring(w.n_trans, w.radius, w.psi0)
    tp = _lib.TraceParams(w.n_rays, w.max_steps(), w.ds, 1500.0)
    return grid, ring, tp


LIB_PATH = None
try:  # path only; loading waits for the first call
    from ._lib import LIB_PATH  # noqa: F401
except Exception:  # torch missing: the binding is unusable anyway
    pass
