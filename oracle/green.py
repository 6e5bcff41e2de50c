"""Ray Green's functions and the reciprocal back-projection operands (oracle; test only).

  * Eq. 2D_greens: g = A exp(i [phi + pi/4]), A_geom = A_tab / sqrt(k0);
  * Eq. phase-discretised: phi = omega T - (pi/2) K (lossless: int k ds = omega T);
  * Eq. greens-time-reversed: reciprocal g_dagger = A^-1 exp(-i [phi + pi/4]);
  * Section 3.4: the angular Jacobian factors |d gamma_e / d e| De (and likewise for r);
  * absorbing media (tables with an absorption integral B): A = A_abs A_geom with
    A_abs = exp(-omega^y B) (Eq. amplitude-abs-discretised), in g and, inverted, in g_dagger.

Readings:
  * the phase is reduced modulo 2 pi in FP64 before the complex exponential;
  * |d gamma(x, e)/d e| De is the central difference a_e(x) = 1/2 |wrap(gamma(x, e+1) -
    gamma(x, e-1))| of the binned ray direction gamma = atan2(u_y, u_x) over neighbouring
    transducers (indices mod N, wrap to (-pi, pi]), one-sided when a neighbour's table is
    invalid at x, zero when both are;
  * the back-projection operands are H = a g_dagger, H_x = H u_x, H_y = H u_y, so that the
    pair weight (1 + u_e . u_r) of the two-way isochron gradient factorises (rank 3);
  * invalid table entries give zero operands.
"""
from __future__ import annotations

import math

import numpy as np

from .binning import Tables
from .lossy import absorption_factor
from .medium import C0


def phase(T, K, omega):
    """phi + pi/4 reduced to [0, 2 pi), FP64 (Eqs. 2D_greens and phase-discretised)."""
    return np.mod(omega * T + math.pi / 4.0 - K * (math.pi / 2.0), 2.0 * math.pi)


def wrap(a):
    """Angle wrapped to (-pi, pi]."""
    return -np.mod(-a + math.pi, 2.0 * math.pi) + math.pi


def angular_weights(tb: Tables) -> np.ndarray:
    """a_e(x): central difference of the ray direction over transducers, shape (N, P_m)."""
    gam = np.arctan2(tb.uy, tb.ux)
    v = tb.valid
    gp, gm = np.roll(gam, -1, axis=0), np.roll(gam, 1, axis=0)   # e+1, e-1
    vp, vm = np.roll(v, -1, axis=0), np.roll(v, 1, axis=0)
    both = 0.5 * np.abs(wrap(gp - gm))
    fwd = np.abs(wrap(gp - gam))
    bwd = np.abs(wrap(gam - gm))
    a = np.where(vp & vm, both, np.where(vp, fwd, np.where(vm, bwd, 0.0)))
    return np.where(v, a, 0.0)


def build_green(tb: Tables, omega: float, c0: float = C0, y=None):
    """G, H, H_x, H_y, each (N, P_m) complex128. y: power-law exponent of lossy tables."""
    k0 = omega / c0
    ph = phase(tb.T, tb.K, omega)
    e = np.exp(1j * ph)
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.where(tb.valid, tb.A / math.sqrt(k0) * e, 0.0)
        gdag = np.where(tb.valid, math.sqrt(k0) / tb.A * np.conj(e), 0.0)
        if tb.B is not None:
            ab = absorption_factor(omega, tb.B, y)
            G = G * ab
            gdag = np.where(tb.valid, gdag / ab, 0.0)
    a = angular_weights(tb)
    H = a * gdag
    return G, H, H * tb.ux, H * tb.uy


def direct_data(tb: Tables, omega: float, c0: float = C0, y=None) -> np.ndarray:
    """Ray Green's function at the receivers g(omega, r, e) (Section 6.3.2), shape (N_e, N_r);
    invalid pairs are zero. y: power-law exponent of lossy tables."""
    k0 = omega / c0
    ph = phase(tb.rx_T, tb.rx_K, omega)
    g = np.where(tb.rx_valid, tb.rx_A / math.sqrt(k0) * np.exp(1j * ph), 0.0)
    if tb.rx_B is not None:
        g = g * absorption_factor(omega, tb.rx_B, y)
    return g
