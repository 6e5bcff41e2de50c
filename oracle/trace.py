"""Paraxial ray tracing by Heun's method (oracle; test infrastructure only).

Follows Section 4 of the paper:
  * Hamiltonian ray equations, Eq. ray-equation-reference: dx/ds = k^-1 kvec,
    dkvec/ds = 1/2 grad k [k^-2 kvec.kvec + 1];
  * paraxial (dynamic) system, Eq. ray-equation-paraxial with the four blocks given after it;
  * Heun's predictor-corrector with the wave-vector normalisations of Algorithm 1 and the
    position step along the normalised mean direction;
  * initial conditions of Section 4.4: dx(s0) = 0 and kvec(s0) . dkvec(s0) = 0;
  * ray sampling of Definition 1: s_i = i ds, last step ds' <= ds landing on the ring;
  * discretised phase (Eq. phase-discretised, trapezoid rule), caustic count from sign
    changes of the ray Jacobian, and the geometric amplitude of Eq.
    amplitude-geom-discretised with the reference amplitude of Eq.
    attenuation_geom_reference at the first sample.

All wave-vector quantities are in units of k0 = omega/c0: for a lossless medium the
wavenumber is k = k0 n, the ray system is homogeneous in k, and the rays do not depend on
omega.

Readings (where the paper is silent):
  * fan instead of ray linking: from each transducer e, n_rays launch angles
    gamma0_j = psi_e + pi + (j + 1/2 - n_rays/2) pi / n_rays cover the inward half-plane;
  * the first paraxial Heun stage uses the state at the start of the step (after the
    normalisation of the wave vector), the second the predictor point x + ds q_x with the
    normalised auxiliary wave vector;
  * dkvec(s0) = n(x_e) (-sin gamma0, cos gamma0), the derivative of kvec(s0) with respect to
    the launch angle, so that J(s) = s in a homogeneous medium;
    J = dx . (-t_y, t_x) with t the unit ray direction;
  * the travel time T = int n ds / c0 by the trapezoid rule on each (partial) step;
  * the last step: when the full step would reach |x| >= R, the step is redone with
    ds' = the distance along the current unit direction to the ring (exact in water);
  * a ray that needs more than max_steps steps is invalid;
  * with an absorption map alpha0_s (Eq. amplitude-abs-discretised), B = int alpha0_s ds
    along the ray by the trapezoid rule at the samples, alpha0_s from the same cubic
    B-spline as the map (value only).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .medium import C0, Grid, Ring, bspline


@dataclasses.dataclass
class RaySamples:
    """Samples of every ray, shape (n_rays_total, max_steps + 1); rows past M are NaN."""

    x: np.ndarray
    y: np.ndarray
    T: np.ndarray       # travel time [s]
    J: np.ndarray       # ray Jacobian dx . n_perp (per unit launch angle) [m]
    K: np.ndarray       # cumulative caustic count (int)
    tx: np.ndarray      # unit ray direction
    ty: np.ndarray
    n: np.ndarray       # refractive index at the sample
    A: np.ndarray       # geometric amplitude times sqrt(k0) (A_geom = A / sqrt(k0))
    M: np.ndarray       # index of the last sample of each ray
    valid: np.ndarray   # ray reached the ring within max_steps
    emitter: np.ndarray  # transducer index of each ray
    ray: np.ndarray      # index of the ray in its transducer's fan
    dkx: np.ndarray = None  # paraxial state, kept for the invariant tests
    dky: np.ndarray = None
    dxx: np.ndarray = None
    dxy: np.ndarray = None
    kx: np.ndarray = None
    ky: np.ndarray = None
    B: np.ndarray = None    # int alpha0 ds from the source (absorption map given), else None


def launch_angles(ring: Ring, emitters, n_rays: int) -> np.ndarray:
    """Open fan over the inward half-plane of each transducer, shape (len(emitters), n_rays)."""
    psi = ring.angles()[np.asarray(emitters)]
    j = np.arange(n_rays)
    return psi[:, None] + math.pi + (j[None, :] + 0.5 - n_rays / 2.0) * math.pi / n_rays


def _paraxial_rhs(n, gx, gy, hxx, hxy, hyy, kx, ky, dxx, dxy, dkx, dky):
    """Right-hand side of Eq. ray-equation-paraxial (k -> n):
    d(dx)/ds = -n^-2 kvec (grad n . dx) + n^-1 dk
    d(dk)/ds = grad^2 n dx - n^-1 grad n (grad n . dx) + n^-2 grad n (kvec . dk)."""
    gdx = gx * dxx + gy * dxy
    kdk = kx * dkx + ky * dky
    qdxx = -gdx / (n * n) * kx + dkx / n
    qdxy = -gdx / (n * n) * ky + dky / n
    qdkx = hxx * dxx + hxy * dxy - gdx / n * gx + kdk / (n * n) * gx
    qdky = hxy * dxx + hyy * dxy - gdx / n * gy + kdk / (n * n) * gy
    return qdxx, qdxy, qdkx, qdky


def heun_step(ns, grid, x, y, kx, ky, dxx, dxy, dkx, dky, h):
    """One step of Algorithm 1 with step length h (array or scalar).

    Returns the new state (x, y, kx, ky, dxx, dxy, dkx, dky)."""
    # reference ray
    n, gx, gy, hxx, hxy, hyy = bspline(ns, grid, x, y)
    kn = np.hypot(kx, ky)
    kx = n * kx / kn
    ky = n * ky / kn
    qxx, qxy = kx / n, ky / n
    qkx, qky = gx, gy
    kpx = kx + h * qkx
    kpy = ky + h * qky
    xp = x + h * qxx
    yp = y + h * qxy
    n2, gx2, gy2, hxx2, hxy2, hyy2 = bspline(ns, grid, xp, yp)
    kpn = np.hypot(kpx, kpy)
    kpx = n2 * kpx / kpn
    kpy = n2 * kpy / kpn
    qxx2, qxy2 = kpx / n2, kpy / n2
    qkx2, qky2 = gx2, gy2
    sx = qxx + qxx2
    sy = qxy + qxy2
    sn = np.hypot(sx, sy)
    x_new = x + h * sx / sn
    y_new = y + h * sy / sn
    kx_new = kx + h * (qkx + qkx2) / 2.0
    ky_new = ky + h * (qky + qky2) / 2.0
    # paraxial ray
    a1, a2, a3, a4 = _paraxial_rhs(n, gx, gy, hxx, hxy, hyy, kx, ky, dxx, dxy, dkx, dky)
    dkpx = dkx + h * a3
    dkpy = dky + h * a4
    dxpx = dxx + h * a1
    dxpy = dxy + h * a2
    b1, b2, b3, b4 = _paraxial_rhs(n2, gx2, gy2, hxx2, hxy2, hyy2, kpx, kpy,
                                   dxpx, dxpy, dkpx, dkpy)
    dxx_new = dxx + h * (a1 + b1) / 2.0
    dxy_new = dxy + h * (a2 + b2) / 2.0
    dkx_new = dkx + h * (a3 + b3) / 2.0
    dky_new = dky + h * (a4 + b4) / 2.0
    return x_new, y_new, kx_new, ky_new, dxx_new, dxy_new, dkx_new, dky_new


def trace(ns: np.ndarray, grid: Grid, ring: Ring, n_rays: int, ds: float, max_steps: int,
          emitters=None, c0: float = C0, angles=None, keep_paraxial: bool = False,
          stop_at_ring: bool = True, alpha=None) -> RaySamples:
    """Trace the fan of every listed transducer through the refractive-index map ns.

    angles: optional launch angles (n_emitters, n_rays_per) overriding the default fan.
    stop_at_ring=False runs exactly max_steps full steps (used by the convergence tests).
    alpha: optional absorption map (ny, nx) whose line integral B is kept per sample.
    """
    if emitters is None:
        emitters = np.arange(ring.n)
    emitters = np.asarray(emitters)
    gam = launch_angles(ring, emitters, n_rays) if angles is None else np.asarray(angles)
    n_per = gam.shape[1]
    gam = gam.ravel()
    em = np.repeat(emitters, n_per)
    rj = np.tile(np.arange(n_per), len(emitters))
    pos = ring.positions()[em]
    R = ring.radius
    nr = gam.size
    S = max_steps + 1

    X = np.full((nr, S), np.nan)
    Y = np.full((nr, S), np.nan)
    T = np.full((nr, S), np.nan)
    J = np.full((nr, S), np.nan)
    Kc = np.zeros((nr, S), dtype=np.int64)
    TX = np.full((nr, S), np.nan)
    TY = np.full((nr, S), np.nan)
    NN = np.full((nr, S), np.nan)
    BB = None if alpha is None else np.full((nr, S), np.nan)
    keep = {}
    if keep_paraxial:
        for key in ("dxx", "dxy", "dkx", "dky", "kx", "ky"):
            keep[key] = np.full((nr, S), np.nan)

    # initial conditions (Section 4.4): x = x_e, kvec = n (cos g, sin g), dx = 0, k . dk = 0
    x = pos[:, 0].copy()
    y = pos[:, 1].copy()
    n0 = bspline(ns, grid, x, y)[0]
    kx = n0 * np.cos(gam)
    ky = n0 * np.sin(gam)
    dxx = np.zeros(nr)
    dxy = np.zeros(nr)
    dkx = -n0 * np.sin(gam)
    dky = n0 * np.cos(gam)
    X[:, 0], Y[:, 0], T[:, 0], J[:, 0] = x, y, 0.0, 0.0
    TX[:, 0], TY[:, 0], NN[:, 0] = np.cos(gam), np.sin(gam), n0
    if alpha is not None:
        BB[:, 0] = 0.0
        al_cur = bspline(alpha, grid, x, y)[0]
    if keep_paraxial:
        for key, val in (("dxx", dxx), ("dxy", dxy), ("dkx", dkx), ("dky", dky),
                         ("kx", kx), ("ky", ky)):
            keep[key][:, 0] = val

    M = np.zeros(nr, dtype=np.int64)
    valid = np.zeros(nr, dtype=bool)
    active = np.arange(nr)
    n_cur = n0.copy()
    for i in range(max_steps):
        if active.size == 0:
            break
        a = active
        st = (x[a], y[a], kx[a], ky[a], dxx[a], dxy[a], dkx[a], dky[a])
        new = heun_step(ns, grid, *st, ds)
        h = np.full(a.size, ds)
        if stop_at_ring:
            out = new[0] ** 2 + new[1] ** 2 >= R * R
            if np.any(out):
                # last step (Definition 1): distance along the unit direction to the ring
                o = np.flatnonzero(out)
                xo, yo = st[0][o], st[1][o]
                kn = np.hypot(st[2][o], st[3][o])
                txo, tyo = st[2][o] / kn, st[3][o] / kn
                b = xo * txo + yo * tyo
                disc = b * b + R * R - (xo * xo + yo * yo)
                hp = -b + np.sqrt(np.maximum(disc, 0.0))
                hp = np.clip(hp, 0.0, ds)
                sub = tuple(s[o] for s in st)
                new_o = heun_step(ns, grid, *sub, hp)
                new = tuple(np.where(out, 0.0, v) for v in new)
                for v, vo in zip(new, new_o):
                    v[o] = vo
                h[o] = hp
        else:
            out = np.zeros(a.size, dtype=bool)
        x[a], y[a], kx[a], ky[a], dxx[a], dxy[a], dkx[a], dky[a] = new
        n_new = bspline(ns, grid, x[a], y[a])[0]
        kn = np.hypot(kx[a], ky[a])
        tx, ty = kx[a] / kn, ky[a] / kn
        X[a, i + 1], Y[a, i + 1] = x[a], y[a]
        # trapezoid rule for T = int n ds / c0 (Eq. phase-discretised / omega)
        T[a, i + 1] = T[a, i] + h * (n_cur[a] + n_new) / (2.0 * c0)
        if alpha is not None:
            # trapezoid rule for B = int alpha0 ds (Eq. amplitude-abs-discretised / omega^y)
            al_new = bspline(alpha, grid, x[a], y[a])[0]
            BB[a, i + 1] = BB[a, i] + h * (al_cur[a] + al_new) / 2.0
            al_cur[a] = al_new
        Jn = dxx[a] * (-ty) + dxy[a] * tx
        J[a, i + 1] = Jn
        # caustic count: sign changes of the Jacobian (Eq. phase-discretised)
        if i >= 1:
            Kc[a, i + 1] = Kc[a, i] + (Jn * J[a, i] < 0.0)
        TX[a, i + 1], TY[a, i + 1], NN[a, i + 1] = tx, ty, n_new
        if keep_paraxial:
            for key, val in (("dxx", dxx), ("dxy", dxy), ("dkx", dkx), ("dky", dky),
                             ("kx", kx), ("ky", ky)):
                keep[key][a, i + 1] = val[a]
        n_cur[a] = n_new
        done = out
        M[a[done]] = i + 1
        valid[a[done]] = True
        active = a[~done]
    if not stop_at_ring:
        M[:] = max_steps
        valid[:] = True

    # geometric amplitude (Eq. amplitude-geom-discretised with Eq. attenuation_geom_reference)
    # A_geom(s_i) = [n(s_1)/n(s_i) J(s_1)/|J(s_i)|]^(1/2) [8 pi k0 |x(s_1) - x(s_0)|]^(-1/2);
    # the stored A is A_geom * sqrt(k0).
    s1 = np.hypot(X[:, 1] - X[:, 0], Y[:, 1] - Y[:, 0])
    with np.errstate(divide="ignore", invalid="ignore"):
        A = np.sqrt(NN[:, 1:2] / NN * J[:, 1:2] / np.abs(J)) / np.sqrt(8.0 * math.pi * s1[:, None])
    A[:, 0] = np.nan
    return RaySamples(x=X, y=Y, T=T, J=J, K=Kc, tx=TX, ty=TY, n=NN, A=A, M=M, valid=valid,
                      emitter=em, ray=rj, B=BB, **keep)
