"""Born forward operator, its adjoint and the Hessian-free back-projection (oracle; test only).

Section 3.1: delta g(omega, r, e)[dm] = int dx' g(omega, r, x') Upsilon_m g(omega, x', e) dm(x')
(Eqs. perturb1, derivative, scattering-potential; lossless Upsilon_m = omega^2).
Discretised over the mask nodes with the node area h^2 (int dx' -> sum h^2); g(r, x') =
g(x', r) by reciprocity, so d[e, r] = sum_p G[e, p] G[r, p] v[p] with v = w dm, w = Upsilon h^2.

Eq. functional-gradient with Q = 1 is the adjoint: grad[p] = Re{ conj(w[p]) sum_{e,r}
conj(G[e,p] G[r,p]) R[e,r] }.

Eqs. sound_speed_update and sound_speed_update2: the Hessian-free search direction
dm(x') = -Re sum_{e,r} Lambda(x') g_res(r, e) with
Lambda = (De Dr Domega / (2 pi)^3) |dgamma_e/de| |dgamma_r/dr| |d|kbar|/domega| |kbar|
         Upsilon_m^-1 g_dagger(x', e) g_dagger(x', r).
Readings:
  * kbar is the gradient of the two-way phase phi(x', e) + phi(r, x'), i.e. k (u_e + u_r)
    with u the direction of the ray from each transducer at x', so |kbar| |d|kbar|/domega| =
    (2 k / c)(1 + u_e . u_r) for a lossless medium (the literal form with k (u_e - u_r) is
    available as isochron_sign = -1);
  * the leading minus sign makes dm a descent direction for g_res = g - data (Eq. residual);
  * Domega is the spacing of the frequency list (omega itself for a single frequency);
  * absorbing media (Section 2.2, Szabo's model): Upsilon_m = omega c k~ is complex, and
    |kbar| |d|kbar|/domega| = 2 k (1 + u_e . u_r) dk/domega with the dispersive k and
    dk/domega = 1/c + y tan(pi y/2) omega^(y-1) alpha0 (Section 3.4), so S is complex and the
    direction takes the real part of S times the complex double sum.
"""
from __future__ import annotations

import math

import numpy as np

from . import lossy


def forward_bruteforce(G, v):
    """d[e, r] = sum_p G[e, p] v[p] G[r, p] as an explicit triple loop (tiny sizes only)."""
    N, P = G.shape
    d = np.zeros((N, N), dtype=np.complex128)
    for e in range(N):
        for r in range(N):
            acc = 0.0 + 0.0j
            for p in range(P):
                acc += G[r, p] * v[p] * G[e, p]
            d[e, r] = acc
    return d


def forward(G, w, delta):
    """Born forward operator: d = G diag(w delta) G^T (complex, no conjugation)."""
    v = np.asarray(w) * np.asarray(delta)
    return (G * v[None, :]) @ G.T


def adjoint(G, w, R):
    """Q = 1 gradient: grad[p] = Re{ conj(w[p]) sum_e conj(G[e,p]) (R conj(G))[e,p] }."""
    Y = R @ np.conj(G)
    return np.real(np.conj(w) * np.sum(np.conj(G) * Y, axis=0))


def backproject_weight(omega, d_omega, c, alpha0=None, y=None):
    """S = (Domega / (2 pi)^3) (2 k dk/domega) / Upsilon_m: lossless (alpha0 None) k = omega/c,
    dk/domega = 1/c, Upsilon_m = omega^2 (real); otherwise the dispersive k, the alpha0 term of
    dk/domega and the complex Upsilon_m = omega c k~ (complex S)."""
    if alpha0 is None:
        k = omega / c
        return d_omega / (2.0 * math.pi) ** 3 * (2.0 * k / c) / omega ** 2
    k = lossy.wavenumber(omega, c, alpha0, y)
    two_k_dk = 2.0 * k / c + 2.0 * k * (y * lossy.tan_py(y) * omega ** (y - 1.0) * alpha0)
    return (d_omega / (2.0 * math.pi) ** 3 * two_k_dk / omega ** 2
            / lossy.relative_potential(omega, c, alpha0, y))


def backproject(R, H, Hx, Hy, S, isochron_sign=1.0):
    """Hessian-free direction, rank-3 form:
    dm[p] = -Re{ S[p] sum_e [H (R H) + s (Hx (R Hx) + Hy (R Hy))][e, p] }."""
    acc = np.sum(H * (R @ H), axis=0)
    acc = acc + isochron_sign * (np.sum(Hx * (R @ Hx), axis=0) + np.sum(Hy * (R @ Hy), axis=0))
    return -np.real(S * acc)


def backproject_literal(R, H, ux, uy, S, isochron_sign=1.0):
    """Same as backproject, as the literal double sum over (e, r) with the pair weight
    (1 + s u_e . u_r) (small sizes only)."""
    N, P = H.shape
    out = np.zeros(P)
    for p in range(P):
        acc = 0.0 + 0.0j
        for e in range(N):
            for r in range(N):
                wgt = 1.0 + isochron_sign * (ux[e, p] * ux[r, p] + uy[e, p] * uy[r, p])
                acc += R[e, r] * H[e, p] * H[r, p] * wgt
        out[p] = -np.real(S[p] * acc)
    return out
