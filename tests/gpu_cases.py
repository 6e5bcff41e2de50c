"""Shared cases and converters for the GPU parity tests (oracle on the host, HIP path on
cuda:0). Inputs come from the seeded phantoms module; expected values only from oracle/."""
import functools
import math

import numpy as np

import phantoms as ph
from oracle import binning
from oracle.medium import Grid, Ring, box_smooth, refractive_index
from oracle.step import StepSetup
from oracle.trace import trace

C0 = 1500.0


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


_PARAMS = {
    # N, R, dx, n_rays, seed, amplitude (m/s), sigma of the inclusion
    "small": (32, 0.02, 0.4e-3, 180, 11, 45.0, 4e-3),
    "ragged": (37, 0.021, 0.37e-3, 101, 12, -30.0, 3e-3),
    # a strong slow lens: rays through it cross (caustics), the fans fold
    "folded": (32, 0.02, 0.4e-3, 180, 14, -300.0, 3e-3),
    # several row slabs of the 16-bit back-projection (256 transducers each), transducer
    # blocks of 64 with a partial last one (300 = 4 x 64 + 44), a partial last node tile
    "wide": (300, 0.021, 0.37e-3, 101, 13, 35.0, 3e-3),
}


@functools.lru_cache(maxsize=None)
def case(name):
    """(StepSetup, c map) of a named parity case."""
    if name == "ring64":
        w = ph.SMALL
        grid = Grid(w.nx, w.ny, w.dx, w.x0, w.y0, w.mask_radius)
        st = StepSetup(grid, Ring(w.n_trans, w.radius), w.n_rays, w.ds, w.max_steps())
        return st, ph.phantom_for(w)
    if name not in _PARAMS:
        raise KeyError(name)
    N, R, dx, nr, seed, amp, sig = _PARAMS[name]
    nx = int(math.ceil(2 * (R + 2e-3) / dx)) + 1
    x0 = -(nx - 1) * dx / 2
    grid = Grid(nx, nx, dx, x0, x0, 0.9 * R)
    st = StepSetup(grid, Ring(N, R), nr, 0.2e-3, int(math.ceil(2.5 * R / 0.2e-3)) + 2)
    c = ph.gaussian_inclusion(nx, nx, dx, x0, x0, seed=seed, amp=amp, sigma=sig,
                              centre_radius=0.3 * R, mask_radius=0.9 * R)
    return st, c


@functools.lru_cache(maxsize=None)
def absorption_case(name, y=1.4):
    """alpha0 (Np (rad/s)^-y m^-1) of a named parity case: a 1 dB MHz^-y cm^-1 peak on the
    case's inclusion (ring64: the absorption of its workload's phantom)."""
    if name == "ring64":
        return ph.absorption_for(ph.SMALL, y=y)
    N, R, dx, nr, seed, amp, sig = _PARAMS[name]
    st, _ = case(name)
    g = st.grid
    a = ph.gaussian_absorption(g.nx, g.ny, g.dx, g.x0, g.y0, seed=seed, amp_db=1.0, sigma=sig,
                               centre_radius=0.3 * R, mask_radius=0.9 * R)
    return ph.db_to_neper(a, y)


def oracle_tables_of(st, ns, emitters=None):
    """Oracle tables of the map the GPU traces: ns rounded to FP32 (the tracer's input).
    Near a focus the amplitude follows the map's second differences closely enough that
    the rounding alone moves it by percents."""
    ns32 = np.asarray(ns, dtype=np.float32).astype(np.float64)
    s = trace(ns32, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, emitters=emitters,
              c0=st.c0)
    return binning.tables(s, st.grid, st.ring, st.ds, st.max_steps, emitters=emitters,
                          c0=st.c0), ns32


@functools.lru_cache(maxsize=None)
def oracle_tables(name, window=1):
    st, c = case(name)
    return oracle_tables_of(st, ns_of(c, window))


def abi_structs(st):
    from paper_2211_00316_amd import _lib

    g = st.grid
    grid = _lib.Grid(g.nx, g.ny, g.dx, g.x0, g.y0, g.mask_radius)
    ring = _lib.Ring(st.ring.n, st.ring.radius, st.ring.psi0)
    tp = _lib.TraceParams(st.n_rays, st.max_steps, st.ds, st.c0)
    return grid, ring, tp


def tables_to_gpu(tb, device="cuda:0"):
    """Oracle tables as the C-ABI table tensors (inputs of the later stages)."""
    import torch
    from paper_2211_00316_amd import _lib

    f = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    flags = np.where(tb.valid, 0x80 | (tb.K & 3), 0).astype(np.uint8)
    rxf = np.where(tb.rx_valid, 0x80 | (tb.rx_K & 3), 0).astype(np.uint8)
    return _lib.Tables(f(tb.T, torch.float64), f(tb.A, torch.float32), f(tb.ux, torch.float32),
                       f(tb.uy, torch.float32), f(flags, torch.uint8), f(tb.rx_T, torch.float64),
                       f(tb.rx_A, torch.float32), f(rxf, torch.uint8))


def to_np(t):
    return t.detach().cpu().numpy()


def ns_of(c, window):
    return box_smooth(refractive_index(c, C0), window)
