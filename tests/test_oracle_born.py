"""Pins of the oracle's Born forward operator, Q=1 adjoint and Hessian-free back-projection
(Section 3, Appendix B, Appendix D)."""
import math

import numpy as np
import pytest
from scipy.special import j0, j1

from oracle import born, green
from tests.oracle_fixtures import C0, water_tables


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_forward_matrix_equals_bruteforce_sum():
    G = _rand((5, 9), 1)
    w = _rand(9, 2)
    delta = np.random.default_rng(3).standard_normal(9)
    ref = born.forward_bruteforce(G, w * delta)
    assert np.max(np.abs(born.forward(G, w, delta) - ref)) < 1e-13 * np.max(np.abs(ref))


def test_forward_is_symmetric_by_reciprocity():
    G = _rand((7, 30), 4)
    d = born.forward(G, np.ones(30), np.random.default_rng(5).standard_normal(30))
    assert np.max(np.abs(d - d.T)) < 1e-13


def test_adjoint_dot_product():
    # <F delta, R> = <delta, F^H R> with <a, b> = Re sum conj(a) b (Eq. functional-gradient, Q=1)
    G = _rand((11, 40), 6)
    w = _rand(40, 7)
    delta = np.random.default_rng(8).standard_normal(40)
    R = _rand((11, 11), 9)
    lhs = np.real(np.vdot(born.forward(G, w, delta), R))
    rhs = np.dot(delta, born.adjoint(G, w, R))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_point_scatterer_closed_form():
    # A single scatterer in water: d[e, r] = g0(r, x_s) omega^2 h^2 dm g0(x_s, e) with the
    # Appendix B Green's function g0 = [8 pi k0 |x - x'|]^-1/2 exp(i (k0 |x - x'| + pi/4)).
    st, tb = water_tables()
    om = 2 * math.pi * 250e3
    k0 = om / C0
    G = green.build_green(tb, om)[0]
    qx, qy = st.grid.mask_coords()
    p = int(np.argmin((qx - 3e-3) ** 2 + (qy + 2e-3) ** 2))
    delta = np.zeros(qx.size)
    delta[p] = 2e-9
    w = np.full(qx.size, om ** 2 * st.grid.dx ** 2)
    d = born.forward(G, w, delta)
    pos = st.ring.positions()
    r = np.hypot(pos[:, 0] - qx[p], pos[:, 1] - qy[p])
    g0 = (8 * math.pi * k0 * r) ** -0.5 * np.exp(1j * (k0 * r + math.pi / 4))
    ref = np.outer(g0, g0) * om ** 2 * st.grid.dx ** 2 * 2e-9
    assert np.max(np.abs(d - ref)) < 1e-10 * np.max(np.abs(ref))


def test_backprojection_rank3_equals_literal_double_sum():
    N, P = 6, 13
    rng = np.random.default_rng(10)
    H = _rand((N, P), 11)
    ang = rng.uniform(0, 2 * math.pi, (N, P))
    ux, uy = np.cos(ang), np.sin(ang)
    R = _rand((N, N), 12)
    S = rng.uniform(0.5, 2.0, P)
    for sgn in (1.0, -1.0):
        a = born.backproject(R, H, H * ux, H * uy, S, sgn)
        b = born.backproject_literal(R, H, ux, uy, S, sgn)
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


@pytest.fixture(scope="module")
def psf_case():
    # Water, ring of 128 at R = 25 mm, f = 300 kHz: 2 k R = 63 < N, so the ring samples the
    # angles finely enough for the change of variables of Section 3.3.
    st, tb = water_tables(N=128, R=0.025, dx=0.25e-3, n_rays=360)
    om = 2 * math.pi * 300e3
    G, H, Hx, Hy = green.build_green(tb, om)
    qx, qy = st.grid.mask_coords()
    p0 = int(np.argmin((qx - 3e-3) ** 2 + (qy + 2e-3) ** 2))
    dm0 = 1e-9
    delta = np.zeros(qx.size)
    delta[p0] = dm0
    w = np.full(qx.size, om ** 2 * st.grid.dx ** 2)
    N = st.ring.n
    R = -born.forward(G, w, delta) * ~np.eye(N, dtype=bool)   # g_res = g_water - data
    S = born.backproject_weight(om, om, np.full(qx.size, C0))
    return dict(st=st, om=om, qx=qx, qy=qy, p0=p0, dm0=dm0, R=R, H=H, Hx=Hx, Hy=Hy, S=S)


def test_point_spread_function_of_one_step(psf_case):
    # Appendix D: at one frequency the preconditioned Hessian kernel is
    # (1/2 pi) 2 k dk [J0^2 - J1^2](k |x - x0|); one step on a point scatterer of strength
    # h^2 dm0 returns that kernel (dk = domega / c0, domega = omega here).
    c = psf_case
    k = c["om"] / C0
    dm = born.backproject(c["R"], c["H"], c["Hx"], c["Hy"], c["S"])
    xd = np.hypot(c["qx"] - c["qx"][c["p0"]], c["qy"] - c["qy"][c["p0"]])
    h2 = c["st"].grid.dx ** 2
    psf = h2 * c["dm0"] * (2 * k * k / (2 * math.pi)) * (j0(k * xd) ** 2 - j1(k * xd) ** 2)
    # peak: exact up to the quadrature error of sum_e a_e u_e (the phases cancel at x0)
    assert abs(dm[c["p0"]] / psf[c["p0"]] - 1) < 0.02
    lam = 2 * math.pi / k
    for rad in (0.5 * lam, lam, 2 * lam):
        sel = xd < rad
        assert np.corrcoef(dm[sel], psf[sel])[0, 1] > 0.999
    # the paper-literal difference form of kbar does not give a delta-like kernel
    dm_lit = born.backproject(c["R"], c["H"], c["Hx"], c["Hy"], c["S"], -1.0)
    sel = xd < 2 * lam
    assert np.corrcoef(dm_lit[sel], psf[sel])[0, 1] < 0.6


def test_step_direction_has_the_scatterer_sign(psf_case):
    # dm = -Re sum Lambda g_res is a descent direction: a positive scatterer is recovered
    # with a positive peak, and the direction correlates positively with the truth.
    c = psf_case
    dm = born.backproject(c["R"], c["H"], c["Hx"], c["Hy"], c["S"])
    assert dm[c["p0"]] > 0
    assert np.argmax(dm) == c["p0"]
