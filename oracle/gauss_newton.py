"""Hessian-based (Gauss-Newton) ray-Born inversion and the prototype Born inversion (oracle;
test infrastructure only).

Section 6.3.2(b): each frequency set's linearised subproblem (Eq. linearised-linearised-
subproblem with Q = 1 for every (omega, r, e, x)) is solved for the perturbation of the
squared slowness by iterating on the actions of the Hessian (Eq. hessian-action) with
conjugate gradients, 10-15 inner iterations whose early end regularises the solution; the
result is a Gauss-Newton direction. Section 6.3.2(c): the prototype Born inversion follows
the same procedure with the Green's functions of water computed analytically (App. B) instead
of traced rays; the sound speed then enters only the scattering potential.

Readings (the paper refers the details to the author's earlier work):
  * the unknown is real, so with J_w the Born operator of Eqs. perturb1 and derivative
    (node weight w = Upsilon_m h^2 = omega^2 h^2, lossless) restricted to the pairs the
    residual keeps (valid, e != r): Hessian action H x = Re sum_w J_w^H J_w x and gradient
    grad = Re sum_w J_w^H g_res,w (Eq. functional-gradient with Q = 1); both are sums of the
    Q = 1 adjoint of oracle.born;
  * conjugate gradients on H x = -grad start at zero and take exactly n_inner iterations
    (fewer only if the residual of the normal equations vanishes); the model update is
    m <- m + tau x (tau = 1: the Gauss-Newton step itself);
  * ray model: tables, Green's functions and predicted data as in the Hessian-free step
    (oracle.step: rays on the smoothed map, the rough part m - m_s in the predicted data);
  * water model (prototype Born): every node and every pair e != r is valid, T = |x - x_e|/c0,
    A = (8 pi |x - x_e|)^-1/2 (A_geom sqrt(k0), the App. B amplitude), u along x - x_e, no
    caustics; predicted data g0(r, e) + F0 (m - c0^-2) (first order about water).
"""
from __future__ import annotations

import math

import numpy as np

from . import born, green
from .binning import Tables
from .step import StepSetup, predicted, residual, tables_for, update


def water_tables(st: StepSetup) -> Tables:
    """Analytic tables of water (straight rays from every transducer)."""
    qx, qy = st.grid.mask_coords()
    pos = st.ring.positions()
    N = st.ring.n
    dx = qx[None, :] - pos[:, 0, None]
    dy = qy[None, :] - pos[:, 1, None]
    d = np.hypot(dx, dy)
    chord = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
    off = ~np.eye(N, dtype=bool)
    safe = np.where(off, chord, 1.0)
    return Tables(valid=np.ones_like(d, dtype=bool), T=d / st.c0,
                  A=(8.0 * math.pi * d) ** -0.5, ux=dx / d, uy=dy / d,
                  K=np.zeros(d.shape, dtype=np.int64), rx_valid=off,
                  rx_T=np.where(off, chord / st.c0, 0.0),
                  rx_A=np.where(off, (8.0 * math.pi * safe) ** -0.5, 0.0),
                  rx_K=np.zeros((N, N), dtype=np.int64))


def jacobian(G, w, keep, x):
    """J x: the Born forward of the perturbation x on the kept pairs (zero elsewhere)."""
    return np.where(keep, born.forward(G, w, x), 0.0)


def normal_apply(ops, x):
    """Hessian action H x = Re sum_w J_w^H J_w x over the frequencies' (G, w, keep)."""
    return sum(born.adjoint(G, w, jacobian(G, w, keep, x)) for G, w, keep in ops)


def gradient(ops, residuals):
    """grad = Re sum_w J_w^H g_res,w (the residuals already zero off the kept pairs)."""
    return sum(born.adjoint(G, w, R) for (G, w, _), R in zip(ops, residuals))


def cg(apply, b, n_iter):
    """Conjugate gradients for apply(x) = b from x = 0: (x, [|r_k|] of each iterate)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    hist = [math.sqrt(rr)]
    for _ in range(n_iter):
        if rr == 0.0:
            break
        Ap = apply(p)
        pAp = float(p @ Ap)
        if not pAp > 0.0:
            break
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        hist.append(math.sqrt(rr))
    return x, hist


def gauss_newton_step(c, st: StepSetup, omegas, data, tau, n_inner, window=1, model="ray",
                      return_parts=False, workers=None, map32=False):
    """One Gauss-Newton update of c (ny, nx) from the data of the frequency set omegas
    (data shape (n_omega, N_e, N_r)): model "ray" (Hessian-based ray-Born) or "water"
    (prototype Born); workers and map32 as in oracle.step.tables_for."""
    q = st.grid.mask_index()
    N = st.ring.n
    if model == "ray":
        tb, ns = tables_for(c, st, window, workers=workers, map32=map32)
    elif model == "water":
        tb = water_tables(st)
        dm_w = 1.0 / c.ravel()[q] ** 2 - 1.0 / st.c0 ** 2
    else:
        raise ValueError(model)
    keep = tb.rx_valid & ~np.eye(N, dtype=bool)
    ops, res = [], []
    for k, om in enumerate(omegas):
        w = np.full(q.size, om ** 2 * st.grid.dx ** 2)
        if model == "ray":
            g, (G, _, _, _) = predicted(tb, c, ns, st, om)
        else:
            G = green.build_green(tb, om, st.c0)[0]
            g = green.direct_data(tb, om, st.c0) + born.forward(G, w, dm_w)
        ops.append((G, w, keep))
        res.append(residual(g, data[k], tb.rx_valid))
    grad = gradient(ops, res)
    x, hist = cg(lambda v: normal_apply(ops, v), -grad, n_inner)
    c_new = update(c, x, tau, st.grid)
    if return_parts:
        return c_new, dict(tables=tb, ops=ops, residuals=res, grad=grad, dm=x, cg=hist)
    return c_new
