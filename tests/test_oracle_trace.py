"""Pins of the oracle's paraxial Heun ray tracer (Section 4, Algorithm 1, Section 5).

Closed forms: straight rays in a homogeneous medium (T = |x - x_e|/c0, J = s, the
reference amplitude of Eq. attenuation_geom_reference continued by Eq.
amplitude-geom-discretised equals the 2D free-space amplitude [8 pi k0 s]^-1/2 of Appendix B);
circular rays in a medium with a linear sound-speed gradient (textbook travel time);
the paraxial Jacobian against finite differences of neighbouring rays (the paper's earlier
method, Section 4.2); the paraxial invariant of Eq. paraxial-condition.
"""
import math

import numpy as np
import pytest

import phantoms as ph
from oracle.medium import Grid, Ring, bspline, refractive_index
from oracle.trace import launch_angles, trace

C0 = 1500.0


def _setup(R=0.02, dx=0.25e-3, margin=2e-3):
    nx = int(math.ceil(2 * (R + margin) / dx)) + 1
    x0 = -(nx - 1) * dx / 2
    return Grid(nx, nx, dx, x0, x0, 0.9 * R)


def test_homogeneous_medium_straight_rays_exact():
    g = _setup()
    ring = Ring(16, 0.02)
    ns = np.ones((g.ny, g.nx))
    s = trace(ns, g, ring, 40, 0.2e-3, 300, emitters=[0, 5])
    assert s.valid.all()
    xe = ring.positions()[s.emitter]
    d = np.hypot(s.x - xe[:, :1], s.y - xe[:, 1:])
    ok = np.isfinite(s.T)
    assert np.max(np.abs(s.T - d / C0)[ok]) * C0 < 1e-14
    assert np.max(np.abs(s.J - d)[ok]) < 1e-14            # J(s) = s
    ok1 = ok.copy()
    ok1[:, 0] = False
    assert np.max(np.abs(s.A * np.sqrt(8 * math.pi * d) - 1.0)[ok1]) < 1e-12
    # every ray ends on the ring (Definition 1) and its last step is not longer than ds
    last = np.arange(s.M.size), s.M
    assert np.max(np.abs(np.hypot(s.x[last], s.y[last]) - 0.02)) < 1e-15
    steps = np.hypot(np.diff(s.x, axis=1), np.diff(s.y, axis=1))
    assert np.nanmax(steps) <= 0.2e-3 * (1 + 1e-12)
    assert np.all(s.K == 0)


def test_launch_fan_covers_inward_half_plane():
    ring = Ring(4, 1.0)
    a = launch_angles(ring, [1], 8)[0]
    psi = ring.angles()[1]
    rel = a - psi - math.pi
    assert np.all(np.abs(rel) < math.pi / 2)
    assert np.allclose(np.diff(a), math.pi / 8)
    assert np.isclose(rel[0], -math.pi / 2 + math.pi / 16)


def test_initial_conditions_of_paraxial_system():
    # Section 4.4: dx(s0) = 0 and kvec(s0) . dk(s0) = 0, |kvec| = n.
    g = _setup()
    ring = Ring(16, 0.02)
    ns = np.ones((g.ny, g.nx))
    s = trace(ns, g, ring, 12, 0.2e-3, 300, emitters=[3], keep_paraxial=True)
    assert np.all(s.dxx[:, 0] == 0) and np.all(s.dxy[:, 0] == 0)
    assert np.max(np.abs(s.kx[:, 0] * s.dkx[:, 0] + s.ky[:, 0] * s.dky[:, 0])) < 1e-15
    assert np.allclose(np.hypot(s.kx[:, 0], s.ky[:, 0]), 1.0)


def _linear_medium(gx=500.0, gy=-200.0, R=0.02, dx=0.125e-3):
    g = _setup(R=R, dx=dx)
    c = ph.linear_gradient(g.nx, g.ny, g.dx, g.x0, g.y0, C0, gx, gy)
    return g, c


def _arccosh_time(c_a, gvec, x, xp):
    """Travel time between x and xp in c = c_a + g . x (circular rays)."""
    gn = math.hypot(*gvec)
    cx = c_a + gvec[0] * x[0] + gvec[1] * x[1]
    cp = c_a + gvec[0] * xp[..., 0] + gvec[1] * xp[..., 1]
    d2 = (xp[..., 0] - x[0]) ** 2 + (xp[..., 1] - x[1]) ** 2
    return np.arccosh(1.0 + gn ** 2 * d2 / (2.0 * cx * cp)) / gn


@pytest.mark.slow
def test_linear_gradient_travel_time_closed_form():
    gvec = (500.0, -200.0)
    g, c = _linear_medium(*gvec)
    ns = refractive_index(c, C0)
    ring = Ring(8, 0.02)
    s = trace(ns, g, ring, 24, 0.2e-3, 400, emitters=[0, 3])
    assert s.valid.all()
    pos = ring.positions()
    err = 0.0
    for row in range(s.M.size):
        e = s.emitter[row]
        m = s.M[row]
        pts = np.stack([s.x[row, 1:m + 1], s.y[row, 1:m + 1]], axis=1)
        Tc = _arccosh_time(C0, gvec, pos[e], pts)
        err = max(err, np.max(np.abs(s.T[row, 1:m + 1] - Tc) / Tc))
    assert err < 1e-6, err


@pytest.mark.slow
def test_heun_second_order_convergence():
    # Self-convergence in ds at a fixed arc length (no partial steps): the error ratio of
    # a second-order scheme is 4 when ds halves.
    gvec = (2000.0, 1000.0)
    g, c = _linear_medium(*gvec, dx=0.25e-3)
    ns = refractive_index(c, C0)
    ring = Ring(8, 0.02)
    L = 0.016
    # central part of the fan, so that every ray stays inside the grid for the whole length
    ang = ring.angles()[1] + math.pi + np.linspace(-0.5, 0.5, 5)[None, :]
    res = {}
    for ds in (1.6e-3, 0.8e-3, 0.4e-3, 0.2e-3):
        n = int(round(L / ds))
        s = trace(ns, g, ring, 5, ds, n, emitters=[1], angles=ang, stop_at_ring=False)
        res[ds] = np.stack([s.x[:, n], s.y[:, n], s.T[:, n] * C0, s.J[:, n]], axis=1)
    e1 = np.max(np.abs(res[1.6e-3] - res[0.8e-3]), axis=0)
    e2 = np.max(np.abs(res[0.8e-3] - res[0.4e-3]), axis=0)
    e3 = np.max(np.abs(res[0.4e-3] - res[0.2e-3]), axis=0)
    assert np.all((3.6 < e1 / e2) & (e1 / e2 < 4.4)), e1 / e2
    assert np.all((3.6 < e2 / e3) & (e2 / e3 < 4.4)), e2 / e3


def test_paraxial_jacobian_matches_neighbouring_ray_differences():
    # Section 4.2: the paraxial ray replaces finite differences of auxiliary rays.
    R = 0.02
    g = _setup(R=R)
    c = ph.gaussian_inclusion(g.nx, g.ny, g.dx, g.x0, g.y0, seed=5, amp=45.0, sigma=4e-3,
                              centre_radius=5e-3, mask_radius=0.9 * R)
    ns = refractive_index(c, C0)
    ring = Ring(8, R)
    base = launch_angles(ring, [2], 16)
    eps = 1e-5
    n = int(1.8 * R / 0.2e-3)
    kw = dict(emitters=[2], stop_at_ring=False)
    s0 = trace(ns, g, ring, 16, 0.2e-3, n, angles=base, **kw)
    sp = trace(ns, g, ring, 16, 0.2e-3, n, angles=base + eps, **kw)
    sm = trace(ns, g, ring, 16, 0.2e-3, n, angles=base - eps, **kw)
    # fixed arc length s_i = i ds for all three rays: dx/dgamma0 ~ central difference
    fdx = (sp.x - sm.x) / (2 * eps)
    fdy = (sp.y - sm.y) / (2 * eps)
    Jfd = fdx * (-s0.ty) + fdy * s0.tx
    sel = np.s_[:, 10:]
    rel = np.abs(Jfd[sel] - s0.J[sel]) / np.abs(s0.J[sel])
    # the inclusion does bend these rays (J differs from s by more than the tolerance)
    assert np.max(np.abs(s0.J[sel] - 0.2e-3 * np.arange(10, n + 1))) > 1e-3 * 0.02
    assert np.max(rel) < 1e-4, np.max(rel)


def test_paraxial_invariant_is_conserved():
    # Eq. paraxial-condition: dH = kvec.dk / k - grad k . dx is zero initially and constant
    # along an exact paraxial solution; the Heun discretisation keeps it to O(ds^2).
    R = 0.02
    g = _setup(R=R)
    c = ph.gaussian_inclusion(g.nx, g.ny, g.dx, g.x0, g.y0, seed=7, amp=45.0, sigma=4e-3,
                              centre_radius=5e-3, mask_radius=0.9 * R)
    ns = refractive_index(c, C0)
    ring = Ring(8, R)
    drift = []
    for ds in (0.4e-3, 0.2e-3, 0.1e-3):
        s = trace(ns, g, ring, 16, ds, 600, emitters=[1], keep_paraxial=True)
        ok = np.isfinite(s.x)
        n, gx, gy = bspline(ns, g, s.x[ok], s.y[ok])[:3]
        kn = np.hypot(s.kx[ok], s.ky[ok])
        dH = (s.kx[ok] * s.dkx[ok] + s.ky[ok] * s.dky[ok]) / kn - (gx * s.dxx[ok] + gy * s.dxy[ok])
        drift.append(np.max(np.abs(dH)))
    # |dk| ~ 1 per radian of launch angle
    assert drift[1] < 5e-4
    assert drift[0] / drift[1] > 3.0 and drift[1] / drift[2] > 3.0, drift
