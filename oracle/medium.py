"""Geometry and medium of the oracle (test infrastructure only).

Problem setting (Section 2.1): a circular ring of point transducers that each emit and
receive, enclosing the region where the sound speed c(x) varies; c0 outside. The unknown is
the squared slowness m = c^-2 (Section 3). Lossless media: the wavenumber is k = omega/c
(Eq. wave-number with alpha0 = 0), so k = k0 * n with the refractive index n = c0/c and
k0 = omega/c0.

Readings where the paper is silent:
  * grid-to-ray interpolation (Section 4.5) uses the uniform cubic B-spline whose control
    points are the grid samples of the refractive index (clamped indices at the border);
    value, gradient and Hessian are the analytic derivatives of that spline;
  * the map the rays are traced on is the refractive index smoothed by an odd box window
    (Section 6.3.2: averaging windows of odd size applied to the wavenumber map), edges
    replicated.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C0 = 1500.0


@dataclasses.dataclass(frozen=True)
class Ring:
    """N point transducers at x_e = R (cos psi_e, sin psi_e), psi_e = psi0 + 2 pi e / N."""

    n: int
    radius: float
    psi0: float = 0.0

    def angles(self) -> np.ndarray:
        return self.psi0 + 2.0 * math.pi * np.arange(self.n) / self.n

    def positions(self) -> np.ndarray:
        a = self.angles()
        return np.stack([self.radius * np.cos(a), self.radius * np.sin(a)], axis=1)


@dataclasses.dataclass(frozen=True)
class Grid:
    """Node (j, i) sits at (x0 + i dx, y0 + j dx); flat index p = j nx + i (x fastest).
    The imaging mask keeps nodes with |x| <= mask_radius (Section 6.3: 90 % of the ring)."""

    nx: int
    ny: int
    dx: float
    x0: float
    y0: float
    mask_radius: float

    def coords(self):
        xs = self.x0 + self.dx * np.arange(self.nx)
        ys = self.y0 + self.dx * np.arange(self.ny)
        return np.meshgrid(xs, ys, indexing="xy")

    def mask(self) -> np.ndarray:
        X, Y = self.coords()
        return X * X + Y * Y <= self.mask_radius ** 2

    def mask_index(self) -> np.ndarray:
        """Flat indices of the mask nodes in ascending order (the compact node list)."""
        return np.flatnonzero(self.mask().ravel())

    def mask_coords(self):
        X, Y = self.coords()
        q = self.mask_index()
        return X.ravel()[q], Y.ravel()[q]


def refractive_index(c: np.ndarray, c0: float = C0) -> np.ndarray:
    """n = c0 / c, so that k = k0 n in a lossless medium (Eq. wave-number, alpha0 = 0)."""
    return c0 / c


def box_smooth(f: np.ndarray, w: int) -> np.ndarray:
    """Separable moving average of odd width w with replicated edges (Section 6.3.2)."""
    if w % 2 != 1 or w < 1:
        raise ValueError("smoothing window must be a positive odd integer")
    if w == 1:
        return f.copy()
    h = w // 2
    out = f
    for axis in (1, 0):
        pad = [(0, 0), (0, 0)]
        pad[axis] = (h, h)
        g = np.pad(out, pad, mode="edge")
        acc = np.zeros_like(out)
        for s in range(w):
            sl = [slice(None), slice(None)]
            sl[axis] = slice(s, s + out.shape[axis])
            acc = acc + g[tuple(sl)]
        out = acc / w
    return out


def _basis(t):
    """Uniform cubic B-spline weights of the four control points iu-1 .. iu+2 at
    fractional offset t in [0, 1), with first and second derivatives."""
    t2 = t * t
    t3 = t2 * t
    s = 1.0 - t
    b = [s ** 3 / 6.0, (3 * t3 - 6 * t2 + 4) / 6.0, (-3 * t3 + 3 * t2 + 3 * t + 1) / 6.0, t3 / 6.0]
    d = [-0.5 * s * s, 0.5 * (3 * t2 - 4 * t), 0.5 * (-3 * t2 + 2 * t + 1), 0.5 * t2]
    dd = [s, 3 * t - 2, 1 - 3 * t, t]
    return b, d, dd


def bspline(f: np.ndarray, grid: Grid, x, y):
    """Value, gradient and Hessian of the cubic B-spline of grid samples f at points (x, y).

    Returns (v, gx, gy, hxx, hxy, hyy), each shaped like x. Physical units: derivatives are
    with respect to metres (Section 4.5: smooth values of k, grad k and grad^2 k off-grid).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    u = (x - grid.x0) / grid.dx
    v = (y - grid.y0) / grid.dx
    iu = np.floor(u)
    iv = np.floor(v)
    bu, du, ddu = _basis(u - iu)
    bv, dv, ddv = _basis(v - iv)
    iu = iu.astype(np.int64)
    iv = iv.astype(np.int64)
    val = np.zeros_like(x)
    gx = np.zeros_like(x)
    gy = np.zeros_like(x)
    hxx = np.zeros_like(x)
    hxy = np.zeros_like(x)
    hyy = np.zeros_like(x)
    for b in range(4):
        jj = np.clip(iv - 1 + b, 0, grid.ny - 1)
        for a in range(4):
            ii = np.clip(iu - 1 + a, 0, grid.nx - 1)
            fab = f[jj, ii]
            val += bu[a] * bv[b] * fab
            gx += du[a] * bv[b] * fab
            gy += bu[a] * dv[b] * fab
            hxx += ddu[a] * bv[b] * fab
            hxy += du[a] * dv[b] * fab
            hyy += bu[a] * ddv[b] * fab
    h = grid.dx
    return val, gx / h, gy / h, hxx / (h * h), hxy / (h * h), hyy / (h * h)
