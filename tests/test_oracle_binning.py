"""Pins of the oracle's ray-to-grid triangulation and receiver tables (Section 4.5, 6.3)."""
import copy
import math

import numpy as np

from oracle import binning
from oracle.trace import trace
from tests.oracle_fixtures import C0, small_setup, water_tables


def test_water_tables_exact_at_nodes():
    # Straight rays: T = |x - x_e|/c0 and A sqrt(k0) = [8 pi |x - x_e|]^-1/2 at every node
    # (Appendix B), because the interpolated residual fields are constant in water.
    st, tb = water_tables()
    qx, qy = st.grid.mask_coords()
    pos = st.ring.positions()
    for e in range(st.ring.n):
        d = np.hypot(qx - pos[e, 0], qy - pos[e, 1])
        v = tb.valid[e]
        assert np.array_equal(v, d >= 2 * st.ds)           # every mask node is covered
        assert np.max(np.abs(tb.T[e][v] - d[v] / C0)) * C0 < 1e-15
        assert np.max(np.abs(tb.A[e][v] * np.sqrt(8 * math.pi * d[v]) - 1)) < 1e-12
        ux, uy = (qx - pos[e, 0]) / d, (qy - pos[e, 1]) / d
        # direction: linear interpolation across a triangle spanning dgamma = pi/n_r in
        # angle and ds in radius; its angular error is below dgamma ds / (2 d) + dgamma^2 / 8
        dg = math.pi / st.n_rays
        bound = dg * st.ds / (2 * d[v]) + dg * dg / 8
        assert np.all(np.hypot(tb.ux[e][v] - ux[v], tb.uy[e][v] - uy[v]) < bound)
        assert np.all(tb.K[e] == 0)


def test_water_receiver_tables_exact():
    st, tb = water_tables()
    pos = st.ring.positions()
    N = st.ring.n
    for e in range(N):
        d = np.hypot(pos[:, 0] - pos[e, 0], pos[:, 1] - pos[e, 1])
        v = tb.rx_valid[e]
        assert not v[e] and v.sum() == N - 1
        assert np.max(np.abs(tb.rx_T[e][v] - d[v] / C0)) * C0 < 1e-15
        assert np.max(np.abs(tb.rx_A[e][v] * np.sqrt(8 * math.pi * d[v]) - 1)) < 1e-12


def _water_samples(st, emitters):
    ns = np.ones((st.grid.ny, st.grid.nx))
    return trace(ns, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, emitters=emitters)


def test_linear_fields_are_interpolated_exactly():
    # Barycentric interpolation reproduces any field linear in (x, y) exactly; plant linear
    # residual fields on the water ray samples and recover them at every covered node.
    st = small_setup(N=16)
    e = 3
    s = _water_samples(st, [e])
    xe, ye = st.ring.positions()[e]
    d = np.hypot(s.x - xe, s.y - ye)
    f_dT = lambda x, y: 1e-7 + 2e-6 * x - 3e-6 * y
    f_L = lambda x, y: -1.5 + 4.0 * x + 1.0 * y
    s2 = copy.copy(s)
    s2.T = f_dT(s.x, s.y) + d / C0
    s2.A = np.exp(f_L(s.x, s.y)) / np.sqrt(d)
    s2.tx = np.full_like(s.x, 0.6) + 0.0 * s.x
    s2.ty = np.full_like(s.x, 0.8)
    f_B = lambda x, y: 0.02 + 0.5 * x - 0.3 * y   # absorption integral (Np (rad/s)^y)
    s2.B = f_B(s.x, s.y)
    valid, T, A, ux, uy, K, B = binning.bin_emitter(s2, e, st.grid, st.ring, st.ds,
                                                    st.max_steps)
    qx, qy = st.grid.mask_coords()
    dq = np.hypot(qx - xe, qy - ye)
    assert valid.sum() > 0.9 * valid.size
    assert np.max(np.abs(T[valid] - (f_dT(qx, qy) + dq / C0)[valid])) < 1e-18
    L = np.log(A[valid] * np.sqrt(dq[valid]))
    assert np.max(np.abs(L - f_L(qx, qy)[valid])) < 1e-12
    assert np.allclose(ux[valid], 0.6, atol=1e-14) and np.allclose(uy[valid], 0.8, atol=1e-14)
    assert np.max(np.abs(B[valid] - f_B(qx, qy)[valid])) < 1e-15
    assert np.all(B[~valid] == 0)


def test_smallest_travel_time_wins_where_sheets_overlap():
    # A folded fan: ray 2 retraces ray 0 with a later arrival. Where the quads (0,1) and
    # (1,2) overlap, the node takes the earlier arrival, i.e. the values of fan {0, 1}.
    st = small_setup(N=16, n_rays=64)
    e = 0
    s = _water_samples(st, [e])
    rows = np.flatnonzero(s.emitter == e)
    pick = rows[[30, 31, 30]]
    def sub(idx, late):
        t = copy.copy(s)
        for k in ("x", "y", "T", "J", "K", "tx", "ty", "n", "A"):
            setattr(t, k, getattr(s, k)[idx].copy())
        t.M, t.valid = s.M[idx].copy(), s.valid[idx].copy()
        t.emitter = np.full(idx.size, e)
        t.ray = np.arange(idx.size)
        if late:
            t.T[2] = t.T[2] + 1e-6
        return t
    folded = binning.bin_emitter(sub(pick, True), e, st.grid, st.ring, st.ds, st.max_steps)
    plain = binning.bin_emitter(sub(pick[:2], False), e, st.grid, st.ring, st.ds, st.max_steps)
    v = plain[0]
    assert v.sum() > 5
    assert np.array_equal(folded[0], v)
    assert np.array_equal(folded[1][v], plain[1][v])


def test_binning_is_deterministic():
    st = small_setup(N=16)
    s = _water_samples(st, [5])
    a = binning.bin_emitter(s, 5, st.grid, st.ring, st.ds, st.max_steps)
    b = binning.bin_emitter(s, 5, st.grid, st.ring, st.ds, st.max_steps)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
