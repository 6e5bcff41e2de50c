"""One Hessian-free frequency step and synthetic data (oracle; test infrastructure only).

Section 3 and Section 6.3.2(a): for the current squared slowness m = c^-2, trace rays on the
(smoothed) wavenumber map, form the Green's functions, predict the data at the receivers,
take the residual g_res = g - data (Eq. residual), back-project it with Lambda
(Eqs. sound_speed_update, sound_speed_update2) summed over the frequencies of the set, and
update m <- m + tau dm, c = m^-1/2 (end of Section 3.4). Outside the mask c = c0 (Section 6.3).

Readings:
  * rays are traced and integrated on the smoothed map n_s; the part of the model the smoothing
    removed, m - m_s with m_s = (n_s/c0)^2, enters the predicted data to first order through
    the Born forward operator with w = omega^2 h^2 ("ray_born"); "ray_only" drops that term.
    With a window of 1 both are the same;
  * emitter-receiver pairs with e = r or without a bracketing ray are masked to zero;
  * absorbing media (an Absorption of alpha0 map and exponent y, oracle.lossy): the rays of
    each frequency are traced on n_omega = box_w(c0/c) + c0 tan(pi y/2) omega^(y-1)
    box_w(alpha0), the tables carry B = int box_w(alpha0) ds, the Born weight is
    w = Upsilon_m h^2 with the complex Upsilon_m = omega c k~ of the model's c and alpha0,
    and the rough part m - m_s keeps m_s = (box_w(c0/c)/c0)^2 (alpha0 is not an unknown).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import binning, born, green, linking, lossy
from .medium import C0, Grid, Ring, box_smooth, refractive_index
from .trace import trace


@dataclasses.dataclass
class StepSetup:
    grid: Grid
    ring: Ring
    n_rays: int
    ds: float
    max_steps: int
    c0: float = C0


def _tables_of_chunk(args):
    traced, al, st, emitters = args
    s = trace(traced, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, emitters=emitters,
              c0=st.c0, alpha=al)
    return binning.tables(s, st.grid, st.ring, st.ds, st.max_steps, emitters=emitters, c0=st.c0)


def tables_for(c: np.ndarray, st: StepSetup, window: int, emitters=None, link=None,
               workers=None, map32=False, absorption=None, omega=None):
    """Trace on box_window(c0/c) and bin; returns (Tables, n_s). link (None, or a dict of
    oracle.linking options): receiver tables from the linked rays instead of the fan's
    interpolation in exit angle. workers > 1: the transducers are traced and binned in that
    many processes, in chunks whose table rows are stacked in order (each row depends on its
    own transducer's rays only, so the tables are the same). map32: the traced map is
    rounded to FP32 first (the representation a device receives it in; everything after is
    FP64), for comparisons with a path that stores the map in FP32. absorption (with the
    frequency omega): the rays follow the dispersive map n_omega and the tables carry the
    absorption integral B; n_s (returned) is the sound-speed part box_w(c0/c) either way."""
    ns = box_smooth(refractive_index(c, st.c0), window)
    traced, al = ns, None
    if absorption is not None:
        if omega is None:
            raise ValueError("lossy tables need the frequency omega")
        al = box_smooth(absorption.alpha0, window)
        traced = lossy.tracing_index(ns, al, omega, absorption.y, st.c0)
    if map32:
        ns = ns.astype(np.float32).astype(np.float64)
        traced = traced.astype(np.float32).astype(np.float64) if al is not None else ns
    if workers and workers > 1 and link is None:
        import concurrent.futures
        import multiprocessing

        em = np.arange(st.ring.n) if emitters is None else np.asarray(emitters)
        chunks = [ch for ch in np.array_split(em, min(len(em), 4 * workers)) if ch.size]
        ctx = multiprocessing.get_context("fork")
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            parts = list(ex.map(_tables_of_chunk, [(traced, al, st, ch) for ch in chunks]))
        cat = {}
        for f in dataclasses.fields(binning.Tables):
            vals = [getattr(t, f.name) for t in parts]
            cat[f.name] = None if vals[0] is None else np.concatenate(vals)
        return binning.Tables(**cat), ns
    s = trace(traced, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, emitters=emitters,
              c0=st.c0, alpha=al)
    tb = binning.tables(s, st.grid, st.ring, st.ds, st.max_steps, emitters=emitters, c0=st.c0)
    if link is not None:
        lk = linking.link_receivers(traced, st.grid, st.ring, st.n_rays, st.ds, st.max_steps,
                                    emitters=emitters, c0=st.c0, fan=s, alpha=al, **link)
        tb = dataclasses.replace(tb, rx_valid=lk.valid, rx_T=lk.T, rx_A=lk.A, rx_K=lk.K,
                                 rx_B=lk.B)
    return tb, ns


def born_weight(c, st: StepSetup, omega: float, absorption=None):
    """w = Upsilon_m h^2 at the mask nodes: omega^2 h^2 (lossless), omega c k~ h^2 (lossy)."""
    q = st.grid.mask_index()
    if absorption is None:
        return np.full(q.size, omega ** 2 * st.grid.dx ** 2)
    ups = lossy.scattering_potential(omega, c.ravel()[q], absorption.alpha0.ravel()[q],
                                     absorption.y)
    return ups * st.grid.dx ** 2


def predicted(tb, c, ns, st: StepSetup, omega: float, mode: str = "ray_born", absorption=None):
    """Predicted data g(m; omega, r, e) and the G operands used for it."""
    y = None if absorption is None else absorption.y
    G, H, Hx, Hy = green.build_green(tb, omega, st.c0, y)
    g = green.direct_data(tb, omega, st.c0, y)
    if mode == "ray_born":
        q = st.grid.mask_index()
        m = 1.0 / c.ravel()[q] ** 2
        ms = (ns.ravel()[q] / st.c0) ** 2
        w = born_weight(c, st, omega, absorption)
        g = g + born.forward(G, w, m - ms)
    elif mode != "ray_only":
        raise ValueError(mode)
    return g, (G, H, Hx, Hy)


def residual(g, data, rx_valid):
    """g_res = g - data on valid pairs with e != r, zero elsewhere (Eq. residual)."""
    N = g.shape[0]
    keep = rx_valid & ~np.eye(N, dtype=bool)
    return np.where(keep, g - data, 0.0)


def update(c: np.ndarray, dm_mask: np.ndarray, tau: float, grid: Grid):
    """m <- m + tau dm on the mask (FP64), c = m^-1/2; unchanged outside."""
    q = grid.mask_index()
    m = 1.0 / c.ravel()[q] ** 2
    m_new = m + tau * dm_mask
    out = c.copy().ravel()
    out[q] = 1.0 / np.sqrt(m_new)
    return out.reshape(c.shape)


def frequency_step(c, st: StepSetup, omegas, d_omegas, data, tau, window=1,
                   mode="ray_born", isochron_sign=1.0, return_parts=False, link=None,
                   workers=None, map32=False, absorption=None):
    """One Hessian-free update of the sound speed c (ny, nx) from the data of the frequency
    set omegas (data shape (n_omega, N_e, N_r)); link, workers, map32 and absorption as in
    tables_for (lossy: the rays are traced again for every frequency)."""
    q = st.grid.mask_index()
    cq = c.ravel()[q]
    aq = None if absorption is None else absorption.alpha0.ravel()[q]
    y = None if absorption is None else absorption.y
    dm = np.zeros(q.size)
    parts = []
    tb = ns = None
    for k, (om, dom) in enumerate(zip(omegas, d_omegas)):
        if tb is None or absorption is not None:
            tb, ns = tables_for(c, st, window, link=link, workers=workers, map32=map32,
                                absorption=absorption, omega=om)
        g, (G, H, Hx, Hy) = predicted(tb, c, ns, st, om, mode, absorption)
        R = residual(g, data[k], tb.rx_valid)
        S = born.backproject_weight(om, dom, cq, aq, y)
        dmk = born.backproject(R, H, Hx, Hy, S, isochron_sign)
        dm += dmk
        parts.append(dict(g=g, R=R, G=G, H=H, Hx=Hx, Hy=Hy, dm=dmk, tables=tb))
    c_new = update(c, dm, tau, st.grid)
    if return_parts:
        return c_new, dict(tables=tb, ns=ns, dm=dm, freqs=parts)
    return c_new


def synthesize(c_true, st: StepSetup, omegas, noise, background="water", window=1,
               noise_level=0.01, workers=None, absorption=None):
    """Synthetic measured data: ray-Born prediction about a background plus noise.

    background="water": g(water) + F[water](m_true - m_water) (first-order data about water);
    background="smooth": the ray_born prediction of c_true with the given window (with
    absorption: of the lossy medium, rays traced per frequency).
    noise: unit complex Gaussian samples of shape (n_omega, N, N); sigma = noise_level times
    the rms of the clean data over valid pairs with e != r."""
    N = st.ring.n
    if absorption is not None and background != "smooth":
        raise ValueError("lossy data are synthesised about the smoothed lossy medium")
    if background == "water":
        cw = np.full_like(c_true, st.c0)
        tb, ns = tables_for(cw, st, 1, workers=workers)
        q = st.grid.mask_index()
        dm = 1.0 / c_true.ravel()[q] ** 2 - 1.0 / st.c0 ** 2
    elif absorption is None:
        tb, ns = tables_for(c_true, st, window, workers=workers)
    out = np.zeros((len(omegas), N, N), dtype=np.complex128)
    for k, om in enumerate(omegas):
        if absorption is not None:
            tb, ns = tables_for(c_true, st, window, workers=workers, absorption=absorption,
                                omega=om)
        keep = tb.rx_valid & ~np.eye(N, dtype=bool)
        if background == "water":
            G, _, _, _ = green.build_green(tb, om, st.c0)
            w = np.full(dm.size, om ** 2 * st.grid.dx ** 2)
            clean = green.direct_data(tb, om, st.c0) + born.forward(G, w, dm)
        else:
            clean, _ = predicted(tb, c_true, ns, st, om, "ray_born", absorption)
        rms = math.sqrt(np.mean(np.abs(clean[keep]) ** 2))
        out[k] = clean + noise_level * rms * noise[k]
    return out
