"""Ray linking of every emitter-receiver pair by the secant method (oracle; test
infrastructure only).

Section 4 of the paper starts each ray at the emitter with the wave vector found by ray
linking, so that the ray meets the receiver; Section 6.3 adjusts the initial direction by
the secant method until the ray crosses the ring at the receiver within a tolerance, and
evaluates the Green's function at the terminal point of the linked ray (Section 5). This
module computes, for every emitter e and receiver r != e, the linked ray's travel time,
amplitude and caustic count at r, as a replacement of the receiver tables that the fan
gives by interpolation in exit angle (oracle.binning.receivers_emitter).

Readings (where the paper is silent):
  * starting points: the two neighbouring fan rays whose exit angles bracket the
    receiver's, the bracket the fan's receiver rule picks (smallest interpolated travel
    time); the paper starts from the previous model's linked direction, which one step does
    not have. A pair without such a bracket is invalid, as for the fan;
  * the unknown is the launch angle gamma; f(gamma) = beta(gamma) - beta_r with beta the
    exit angle measured from psi_e in [0, 2 pi) and beta_r = 2 pi ((r - e) mod N) / N;
  * safeguarded secant: the secant point of the last two iterates is taken when it lies
    strictly inside the current bracket (which always holds a sign change of f), otherwise
    the bracket's midpoint; every traced ray narrows the bracket;
  * stop when |f| <= tol or after max_iter traced rays; the traced ray with the smallest
    |f| is the linked ray, valid if |f| <= accept (else the pair is invalid);
  * the rays are traced exactly as the fan's (oracle.trace.trace: Algorithm 1 with the
    paraxial system, Definition 1's last step), so T, A and K at the terminal sample follow
    Eqs. phase-discretised and amplitude-geom-discretised, and with an absorption map the
    absorption integral B of Eq. amplitude-abs-discretised as well.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .medium import C0, Grid, Ring
from .trace import launch_angles, trace

TOL = 1e-9        # radians of exit angle: stop
ACCEPT = 1e-6     # radians: a linked ray further from its receiver is not accepted
MAX_ITER = 12     # traced rays per pair


@dataclasses.dataclass
class Linked:
    """Receiver tables of the linked rays, shape (n_emitters, N)."""

    valid: np.ndarray
    T: np.ndarray
    A: np.ndarray
    K: np.ndarray
    gamma: np.ndarray     # launch angle of the linked ray
    miss: np.ndarray      # |beta - beta_r| of the linked ray (radians)
    rays: np.ndarray      # rays traced by the secant iteration
    B: np.ndarray = None  # absorption integral at the receiver (absorption map given)


def _exit(s, rows, psi_e):
    """Exit angle from psi_e in [0, 2 pi), T, A, K, B (or None) at the terminal sample of
    each row."""
    M = s.M[rows]
    ok = s.valid[rows]
    m = np.where(ok, M, 0)
    x = s.x[rows, m]
    y = s.y[rows, m]
    beta = np.mod(np.arctan2(y, x) - psi_e, 2.0 * math.pi)
    B = None if s.B is None else s.B[rows, m]
    return (ok, np.where(ok, beta, np.nan), s.T[rows, m], s.A[rows, m], s.K[rows, m], B)


def fan_brackets(s, e: int, ring: Ring, c0: float = C0):
    """For each receiver r: the fan ray index j of the bracket (j, j+1) that the fan's
    receiver rule picks (smallest interpolated travel time, lowest j on a tie), -1 if none;
    with the exit angles of the fan."""
    rows = np.flatnonzero(s.emitter == e)
    rows = rows[np.argsort(s.ray[rows])]
    N = ring.n
    psi_e = ring.angles()[e]
    ok, beta, Tm, _, _, _ = _exit(s, rows, psi_e)
    xe, ye = ring.positions()[e]
    m = np.where(ok, s.M[rows], 0)
    dm = np.hypot(s.x[rows, m] - xe, s.y[rows, m] - ye)
    dTm = Tm - dm / c0
    jsel = np.full(N, -1)
    for r in range(N):
        if r == e:
            continue
        br = 2.0 * math.pi * ((r - e) % N) / N
        b0, b1 = beta[:-1], beta[1:]
        pair = ok[:-1] & ok[1:] & (b0 != b1)
        pair &= (np.minimum(b0, b1) <= br) & (br <= np.maximum(b0, b1))
        js = np.flatnonzero(pair)
        if js.size:
            lam = (br - b0[js]) / (b1[js] - b0[js])
            dT = (1.0 - lam) * dTm[js] + lam * dTm[js + 1]
            jsel[r] = js[int(np.argmin(dT))]
    return jsel, beta


def link_emitter(ns: np.ndarray, grid: Grid, ring: Ring, n_rays: int, ds: float,
                 max_steps: int, e: int, c0: float = C0, tol: float = TOL,
                 accept: float = ACCEPT, max_iter: int = MAX_ITER, fan=None, alpha=None):
    """Linked receiver tables of emitter e: (valid, T, A, K, gamma, miss, rays, B), each
    [N]; B (absorption integral) is None without an absorption map alpha."""
    N = ring.n
    if fan is None:
        fan = trace(ns, grid, ring, n_rays, ds, max_steps, emitters=[e], c0=c0, alpha=alpha)
    jsel, beta = fan_brackets(fan, e, ring, c0)
    gam_fan = launch_angles(ring, [e], n_rays)[0]
    psi_e = ring.angles()[e]
    br = 2.0 * math.pi * ((np.arange(N) - e) % N) / N
    act = np.flatnonzero(jsel >= 0)
    # bracket [lo, hi] in gamma with f(lo), f(hi) of opposite sign (or zero); the last two
    # iterates start at the bracket's ends
    lo = gam_fan[jsel[act]]
    hi = gam_fan[jsel[act] + 1]
    flo = beta[jsel[act]] - br[act]
    fhi = beta[jsel[act] + 1] - br[act]
    xp, fp = lo.copy(), flo.copy()
    xc, fc = hi.copy(), fhi.copy()
    best_g = np.full(act.size, np.nan)   # launch angle, |f| and (T, A, K) of the traced ray
    best_f = np.full(act.size, np.inf)   # closest to its receiver
    best = [None] * N
    rays = np.zeros(N, dtype=np.int64)
    open_ = np.ones(act.size, dtype=bool)
    for _ in range(max_iter):
        todo = np.flatnonzero(open_ & (best_f > tol))
        if todo.size == 0:
            break
        den = fc[todo] - fp[todo]
        with np.errstate(divide="ignore", invalid="ignore"):
            cand = xc[todo] - fc[todo] * (xc[todo] - xp[todo]) / den
        a = np.minimum(lo[todo], hi[todo])
        b = np.maximum(lo[todo], hi[todo])
        inside = np.isfinite(cand) & (cand > a) & (cand < b)
        cand = np.where(inside, cand, 0.5 * (lo[todo] + hi[todo]))
        s = trace(ns, grid, ring, n_rays, ds, max_steps, emitters=[e], c0=c0,
                  angles=cand[None, :], alpha=alpha)
        ok, bet, T, A, K, Bx = _exit(s, np.arange(todo.size), psi_e)
        for t, idx in enumerate(todo):
            r = act[idx]
            rays[r] += 1
            if not ok[t]:
                open_[idx] = False   # a ray that does not reach the ring ends the pair
                continue
            f = bet[t] - br[r]
            if abs(f) < best_f[idx]:
                best_f[idx] = abs(f)
                best_g[idx] = cand[t]
                best[r] = (T[t], A[t], K[t], 0.0 if Bx is None else Bx[t])
            # keep the sign change inside the bracket
            if (f < 0) == (flo[idx] < 0):
                lo[idx], flo[idx] = cand[t], f
            else:
                hi[idx], fhi[idx] = cand[t], f
            xp[idx], fp[idx] = xc[idx], fc[idx]
            xc[idx], fc[idx] = cand[t], f
    valid = np.zeros(N, dtype=bool)
    Tout = np.zeros(N)
    Aout = np.zeros(N)
    Kout = np.zeros(N, dtype=np.int64)
    Bout = None if alpha is None else np.zeros(N)
    gam = np.full(N, np.nan)
    miss = np.full(N, np.nan)
    for idx, r in enumerate(act):
        miss[r] = best_f[idx]
        gam[r] = best_g[idx]
        if best[r] is not None and best_f[idx] <= accept:
            valid[r] = True
            Tout[r], Aout[r], Kout[r] = best[r][:3]
            if Bout is not None:
                Bout[r] = best[r][3]
    return valid, Tout, Aout, Kout, gam, miss, rays, Bout


def link_receivers(ns, grid: Grid, ring: Ring, n_rays: int, ds: float, max_steps: int,
                   emitters=None, c0: float = C0, fan=None, **kw) -> Linked:
    """Linked receiver tables of the listed emitters (all by default). fan: the traced fan
    of these emitters, if at hand (else traced per emitter)."""
    if emitters is None:
        emitters = np.arange(ring.n)
    out = [link_emitter(ns, grid, ring, n_rays, ds, max_steps, int(e), c0, fan=fan, **kw)
           for e in emitters]
    st = lambda k: np.stack([o[k] for o in out])
    return Linked(valid=st(0), T=st(1), A=st(2), K=st(3), gamma=st(4), miss=st(5),
                  rays=st(6), B=None if out[0][7] is None else st(7))
