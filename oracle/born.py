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
  * Domega is the spacing of the frequency list (omega itself for a single frequency).
"""
from __future__ import annotations

import math

import numpy as np


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


def backproject_weight(omega, d_omega, c):
    """S = (Domega / (2 pi)^3) (2 k / c) / Upsilon_m with k = omega / c, Upsilon_m = omega^2."""
    k = omega / c
    return d_omega / (2.0 * math.pi) ** 3 * (2.0 * k / c) / omega ** 2


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
