"""Ray-to-grid interpolation and receiver tables (oracle; test infrastructure only).

Section 4.5 and Section 6.3: the Green's-function parameters known on the sampled rays are
carried to the grid nodes by triangulating the sampled ray points and interpolating linearly
inside each triangle; the Green's function at the receivers is obtained from the rays that
reach the ring.

Readings (the paper gives no further detail):
  * for each transducer, the quad between neighbouring rays j, j+1 and samples i, i+1
    (1 <= i < min(M_j, M_j+1)) is split along the (j,i)-(j+1,i+1) diagonal into two triangles;
    quads touching the source sample i = 0 are skipped;
  * the interpolated fields are the smooth residual fields dT = T - |x - x_e|/c0,
    L = ln A + 1/2 ln |x - x_e| and the unit direction t; the caustic count of a triangle is
    the largest of its vertices';
  * a node is covered by a triangle when its three barycentric coordinates are >= -1e-12;
    when several triangles cover a node, the smallest interpolated travel time wins, ties to
    the lowest triangle id ((j (max_steps+1) + i) 2 + half); a node is invalid when no
    triangle covers it or when it lies within 2 ds of the source;
  * receivers: the exit angle of each ray, measured from the source angle in [0, 2 pi), is
    linearly interpolated between neighbouring rays that bracket the receiver angle (dT and L
    interpolated), the smallest travel time wins, and an unbracketed pair is invalid;
  * with an absorption integral B on the rays (Eq. amplitude-abs-discretised), B is carried
    to the nodes and receivers by the same interpolation as dT (it is smooth and zero at the
    source).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .medium import C0, Grid, Ring
from .trace import RaySamples


@dataclasses.dataclass
class Tables:
    """Per-transducer grid tables over the mask nodes, shape (N, P_m), and receiver tables
    shape (N, N) (row = emitter)."""

    valid: np.ndarray
    T: np.ndarray
    A: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    K: np.ndarray
    rx_valid: np.ndarray
    rx_T: np.ndarray
    rx_A: np.ndarray
    rx_K: np.ndarray
    B: np.ndarray = None      # int alpha0 ds of the ray at the node (lossy tables), else None
    rx_B: np.ndarray = None   # the same at the receivers


def _ray_block(s: RaySamples, e: int):
    rows = np.flatnonzero(s.emitter == e)
    order = np.argsort(s.ray[rows])
    return rows[order]


def bin_emitter(s: RaySamples, e: int, grid: Grid, ring: Ring, ds: float, max_steps: int,
                c0: float = C0):
    """Grid tables of transducer e over the mask nodes."""
    rows = _ray_block(s, e)
    xe, ye = ring.positions()[e]
    X, Y = s.x[rows], s.y[rows]
    d = np.hypot(X - xe, Y - ye)
    dT = s.T[rows] - d / c0
    with np.errstate(divide="ignore", invalid="ignore"):
        L = np.log(s.A[rows]) + 0.5 * np.log(d)
    TX, TY, KK = s.tx[rows], s.ty[rows], s.K[rows]
    lossy = s.B is not None
    fields = (("dT", dT), ("L", L), ("tx", TX), ("ty", TY))
    if lossy:
        fields = fields + (("B", s.B[rows]),)
    M = s.M[rows]
    ok = s.valid[rows]
    nr = rows.size

    # triangle list
    tri_j, tri_i = [], []
    for j in range(nr - 1):
        if not (ok[j] and ok[j + 1]):
            continue
        top = min(M[j], M[j + 1])
        ii = np.arange(1, top)
        tri_j.append(np.full(ii.size, j))
        tri_i.append(ii)
    P = grid.nx * grid.ny
    mask_flat = grid.mask().ravel()
    qmap = -np.ones(P, dtype=np.int64)
    qidx = grid.mask_index()
    qmap[qidx] = np.arange(qidx.size)
    Pm = qidx.size
    out_valid = np.zeros(Pm, dtype=bool)
    out = {k: np.zeros(Pm) for k, _ in fields}
    out_K = np.zeros(Pm, dtype=np.int64)
    if not tri_j:
        return _finish(out_valid, out, out_K, grid, xe, ye, ds, c0)
    tj = np.concatenate(tri_j)
    ti = np.concatenate(tri_i)
    # vertices of the two halves
    va = [(tj, ti), (tj + 1, ti), (tj + 1, ti + 1)]
    vb = [(tj, ti), (tj + 1, ti + 1), (tj, ti + 1)]
    cand_node, cand_dT, cand_id, cand_vals = [], [], [], []
    for half, verts in ((0, va), (1, vb)):
        ax, ay = X[verts[0]], Y[verts[0]]
        bx, by = X[verts[1]], Y[verts[1]]
        cx, cy = X[verts[2]], Y[verts[2]]
        # node-index coordinates
        au, av = (ax - grid.x0) / grid.dx, (ay - grid.y0) / grid.dx
        bu, bv = (bx - grid.x0) / grid.dx, (by - grid.y0) / grid.dx
        cu, cv = (cx - grid.x0) / grid.dx, (cy - grid.y0) / grid.dx
        area = (bu - au) * (cv - av) - (bv - av) * (cu - au)
        good = np.abs(area) > 1e-300
        i0 = np.ceil(np.minimum(np.minimum(au, bu), cu)).astype(np.int64)
        i1 = np.floor(np.maximum(np.maximum(au, bu), cu)).astype(np.int64)
        j0 = np.ceil(np.minimum(np.minimum(av, bv), cv)).astype(np.int64)
        j1 = np.floor(np.maximum(np.maximum(av, bv), cv)).astype(np.int64)
        i0 = np.maximum(i0, 0)
        j0 = np.maximum(j0, 0)
        i1 = np.minimum(i1, grid.nx - 1)
        j1 = np.minimum(j1, grid.ny - 1)
        ni = np.maximum(i1 - i0 + 1, 0)
        nj = np.maximum(j1 - j0 + 1, 0)
        cnt = np.where(good, ni * nj, 0)
        tot = int(cnt.sum())
        if tot == 0:
            continue
        t_of = np.repeat(np.arange(cnt.size), cnt)
        start = np.cumsum(cnt) - cnt
        local = np.arange(tot) - start[t_of]
        nii = i0[t_of] + local % ni[t_of]
        njj = j0[t_of] + local // ni[t_of]
        pu = nii.astype(np.float64)
        pv = njj.astype(np.float64)
        A_ = area[t_of]
        la = ((bu[t_of] - pu) * (cv[t_of] - pv) - (bv[t_of] - pv) * (cu[t_of] - pu)) / A_
        lb = ((cu[t_of] - pu) * (av[t_of] - pv) - (cv[t_of] - pv) * (au[t_of] - pu)) / A_
        lc = ((au[t_of] - pu) * (bv[t_of] - pv) - (av[t_of] - pv) * (bu[t_of] - pu)) / A_
        inside = (la >= -1e-12) & (lb >= -1e-12) & (lc >= -1e-12)
        flat = njj * grid.nx + nii
        inside &= mask_flat[flat]
        sel = np.flatnonzero(inside)
        t_sel = t_of[sel]
        lam = (la[sel], lb[sel], lc[sel])
        vals = {}
        for key, fld in fields:
            vals[key] = sum(l * fld[v[0][t_sel], v[1][t_sel]] for l, v in zip(lam, verts))
        kmax = np.maximum(np.maximum(KK[verts[0][0][t_sel], verts[0][1][t_sel]],
                                     KK[verts[1][0][t_sel], verts[1][1][t_sel]]),
                          KK[verts[2][0][t_sel], verts[2][1][t_sel]])
        vals["K"] = kmax
        tid = (tj[t_sel] * (max_steps + 1) + ti[t_sel]) * 2 + half
        cand_node.append(qmap[flat[sel]])
        cand_dT.append(vals["dT"])
        cand_id.append(tid)
        cand_vals.append(vals)
    if cand_node:
        node = np.concatenate(cand_node)
        cdT = np.concatenate(cand_dT)
        cid = np.concatenate(cand_id)
        allv = {k: np.concatenate([v[k] for v in cand_vals]) for k in cand_vals[0]}
        # smallest travel time per node, ties to the lowest triangle id
        order = np.lexsort((cid, cdT, node))
        node_s = node[order]
        first = np.ones(node_s.size, dtype=bool)
        first[1:] = node_s[1:] != node_s[:-1]
        win = order[first]
        q = node[win]
        out_valid[q] = True
        for k, _ in fields:
            out[k][q] = allv[k][win]
        out_K[q] = allv["K"][win]
    return _finish(out_valid, out, out_K, grid, xe, ye, ds, c0)


def _finish(valid, vals, K, grid, xe, ye, ds, c0):
    qx, qy = grid.mask_coords()
    d = np.hypot(qx - xe, qy - ye)
    valid = valid & (d >= 2.0 * ds)
    T = np.where(valid, vals["dT"] + d / c0, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        A = np.where(valid, np.exp(vals["L"]) / np.sqrt(d), 0.0)
        tn = np.hypot(vals["tx"], vals["ty"])
        ux = np.where(valid, vals["tx"] / tn, 0.0)
        uy = np.where(valid, vals["ty"] / tn, 0.0)
    B = np.where(valid, vals["B"], 0.0) if "B" in vals else None
    return valid, T, A, ux, uy, np.where(valid, K, 0), B


def receivers_emitter(s: RaySamples, e: int, ring: Ring, c0: float = C0):
    """Receiver tables of emitter e: (valid, T, A, K, B) for every receiver r (r = e invalid);
    B is None without an absorption integral on the rays."""
    rows = _ray_block(s, e)
    N = ring.n
    pos = ring.positions()
    xe, ye = pos[e]
    ok = s.valid[rows]
    M = s.M[rows]
    xm = np.where(ok, s.x[rows, np.where(ok, M, 0)], np.nan)
    ym = np.where(ok, s.y[rows, np.where(ok, M, 0)], np.nan)
    Tm = np.where(ok, s.T[rows, np.where(ok, M, 0)], np.nan)
    Am = np.where(ok, s.A[rows, np.where(ok, M, 0)], np.nan)
    Km = np.where(ok, s.K[rows, np.where(ok, M, 0)], 0)
    lossy = s.B is not None
    Bm = np.where(ok, s.B[rows, np.where(ok, M, 0)], np.nan) if lossy else None
    dm = np.hypot(xm - xe, ym - ye)
    dTm = Tm - dm / c0
    with np.errstate(divide="ignore", invalid="ignore"):
        Lm = np.log(Am) + 0.5 * np.log(dm)
    beta = np.mod(np.arctan2(ym, xm) - ring.angles()[e], 2.0 * math.pi)
    valid = np.zeros(N, dtype=bool)
    T = np.zeros(N)
    A = np.zeros(N)
    K = np.zeros(N, dtype=np.int64)
    B = np.zeros(N) if lossy else None
    for r in range(N):
        if r == e:
            continue
        br = 2.0 * math.pi * ((r - e) % N) / N
        b0, b1 = beta[:-1], beta[1:]
        pair = ok[:-1] & ok[1:] & (b0 != b1)
        pair &= (np.minimum(b0, b1) <= br) & (br <= np.maximum(b0, b1))
        best = None
        js = np.flatnonzero(pair)
        if js.size:
            lam = (br - b0[js]) / (b1[js] - b0[js])
            dT = (1.0 - lam) * dTm[js] + lam * dTm[js + 1]
            w = int(np.argmin(dT))  # first minimum = lowest ray index on a tie
            L = (1.0 - lam[w]) * Lm[js[w]] + lam[w] * Lm[js[w] + 1]
            Bw = (1.0 - lam[w]) * Bm[js[w]] + lam[w] * Bm[js[w] + 1] if lossy else None
            best = (dT[w], L, max(Km[js[w]], Km[js[w] + 1]), Bw)
        if best is not None:
            dist = math.hypot(pos[r, 0] - xe, pos[r, 1] - ye)
            valid[r] = True
            T[r] = best[0] + dist / c0
            A[r] = math.exp(best[1]) / math.sqrt(dist)
            K[r] = best[2]
            if lossy:
                B[r] = best[3]
    return valid, T, A, K, B


def tables(s: RaySamples, grid: Grid, ring: Ring, ds: float, max_steps: int,
           emitters=None, c0: float = C0) -> Tables:
    """Grid and receiver tables of the listed transducers (all by default)."""
    if emitters is None:
        emitters = np.arange(ring.n)
    rows = []
    rx = []
    for e in emitters:
        rows.append(bin_emitter(s, int(e), grid, ring, ds, max_steps, c0))
        rx.append(receivers_emitter(s, int(e), ring, c0))
    st = lambda k: np.stack([r[k] for r in rows])
    sr = lambda k: np.stack([r[k] for r in rx])
    lossy = s.B is not None
    return Tables(valid=st(0), T=st(1), A=st(2), ux=st(3), uy=st(4), K=st(5),
                  rx_valid=sr(0), rx_T=sr(1), rx_A=sr(2), rx_K=sr(3),
                  B=st(6) if lossy else None, rx_B=sr(4) if lossy else None)
