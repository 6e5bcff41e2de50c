"""Pins of the oracle's lossy, dispersive path (Szabo's model; Section 2.2, Eqs.
szabo_dispersion_equation, wave-number, complex-wavevector, scattering-potential; Section 3.4's
d|kbar|/domega; Section 5, Eq. amplitude-abs-discretised).

What fixes the expected values here, independently of the oracle's own expressions:
  * the other form of Eq. szabo_dispersion_equation, with (-i)^(y+1) evaluated by complex
    arithmetic;
  * derivatives by finite differences: Upsilon_m = d(k~^2)/dm (the coefficient of m in the
    lossy Helmholtz operator) and dk/domega;
  * closed forms in a homogeneous absorbing medium (straight rays, A_abs = exp(-alpha d),
    phase k d with the dispersive k) and in a medium whose dispersion cancels its sound-speed
    gradient at one frequency (straight rays there, line integral of a linear alpha0);
  * the point-spread function of one step (Appendix D) with the dispersive k and dk, whose
    peak is exact because the back-projection inverts the absorption along both rays;
  * alpha0 = 0 reproduces the lossless oracle bit for bit.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import j0, j1

import phantoms as ph
from oracle import born, green, lossy, step
from oracle.linking import link_receivers
from oracle.medium import Grid, Ring
from oracle.trace import trace
from tests.oracle_fixtures import C0, small_setup

Y = 1.4


def test_szabo_second_form_equals_the_first():
    # omega/c - alpha0 (-i)^(y+1) omega^y / cos(pi y / 2) = omega/c + alpha [tan(pi y/2) + i]
    rng = np.random.default_rng(1)
    for y in (1.05, 1.4, 1.5, 1.9, 0.6):
        om = rng.uniform(2e5, 1e7, 20)
        c = rng.uniform(1400.0, 1600.0, 20)
        a0 = ph.db_to_neper(rng.uniform(0.0, 2.0, 20), y)
        first = om / c - a0 * (-1j) ** (y + 1.0) * om ** y / math.cos(math.pi * y / 2.0)
        second = lossy.complex_wavenumber(om, c, a0, y)
        assert np.max(np.abs(second - first) / np.abs(first)) < 1e-13
        # its imaginary part is the power-law absorption alpha0 omega^y
        assert np.allclose(second.imag, a0 * om ** y, rtol=1e-13, atol=0)


def test_tissue_dispersion_raises_the_phase_speed_with_frequency():
    # 1 < y < 2: tan(pi y/2) < 0, so c_p = omega / k grows with omega (Eq. wave-number).
    c, a0 = 1540.0, ph.db_to_neper(0.75, Y)
    om = 2 * math.pi * np.array([0.1e6, 0.5e6, 1.0e6, 2.0e6])
    cp = om / lossy.wavenumber(om, c, a0, Y)
    assert np.all(np.diff(cp) > 0) and np.all(cp > c)


def test_scattering_potential_is_the_m_derivative_of_k_squared():
    # The lossy Helmholtz operator is k~(m)^2 + laplacian with k~ = omega m^1/2 + alpha0 omega^y
    # (tan + i); its derivative with respect to m is the scattering potential omega c k~.
    for om, c, adb in ((2 * math.pi * 3e5, 1480.0, 0.3), (2 * math.pi * 1.2e6, 1570.0, 1.0)):
        a0 = ph.db_to_neper(adb, Y)
        m = c ** -2
        h = 1e-6 * m
        k2 = lambda mm: lossy.complex_wavenumber(om, mm ** -0.5, a0, Y) ** 2
        fd = (k2(m + h) - k2(m - h)) / (2 * h)
        ups = lossy.scattering_potential(om, c, a0, Y)
        assert abs(ups - fd) / abs(ups) < 1e-8
        assert ups.imag > 0                       # absorption: positive imaginary part
    assert lossy.scattering_potential(5.0, 1500.0, 0.0, Y) == 25.0


def test_dk_domega_is_the_frequency_derivative_of_k():
    # Section 3.4: d|kbar|/domega = 2 |cos(theta/2)| dk/domega.
    c, a0 = 1520.0, ph.db_to_neper(0.9, Y)
    for om in 2 * math.pi * np.array([2e5, 8e5, 1.5e6]):
        h = 1e-5 * om
        fd = (lossy.wavenumber(om + h, c, a0, Y) - lossy.wavenumber(om - h, c, a0, Y)) / (2 * h)
        assert abs(lossy.dk_domega(om, c, a0, Y) - fd) < 1e-9 * abs(fd)
        th = 0.7
        kb = lambda w: 2 * lossy.wavenumber(w, c, a0, Y) * abs(math.cos(th / 2))
        fdb = (kb(om + h) - kb(om - h)) / (2 * h)
        assert abs(2 * abs(math.cos(th / 2)) * lossy.dk_domega(om, c, a0, Y) - fdb) < 1e-9 * fdb


def _homogeneous(st, adb):
    a0 = ph.db_to_neper(adb, Y)
    c = np.full((st.grid.ny, st.grid.nx), C0)
    return c, a0, lossy.Absorption(np.full_like(c, a0), Y)


def test_absorption_integral_on_straight_rays_is_exact():
    # Homogeneous absorbing medium: straight rays, B = alpha0 s at every sample (the trapezoid
    # rule and the spline are exact for a constant), and the travel time is s / c_p.
    st = small_setup(N=8, n_rays=40)
    c, a0, ab = _homogeneous(st, 1.0)
    om = 2 * math.pi * 6e5
    n_om = lossy.tracing_index(np.ones_like(c), ab.alpha0, om, Y, C0)
    s = trace(n_om, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, emitters=[0, 3],
              alpha=ab.alpha0)
    pos = st.ring.positions()[s.emitter]
    d = np.hypot(s.x - pos[:, :1], s.y - pos[:, 1:2])
    ok = np.isfinite(d)
    assert np.all(s.valid)
    assert np.max(np.abs(s.B[ok] - a0 * d[ok])) < 1e-12 * a0 * np.max(d[ok])
    kp = lossy.wavenumber(om, C0, a0, Y)
    assert np.max(np.abs(s.T[ok] * om - kp * d[ok])) < 1e-9 * kp * np.max(d[ok])


def test_homogeneous_lossy_green_closed_form():
    # g = [8 pi k0 d]^-1/2 exp(i (k d + pi/4)) exp(-alpha d): the reference amplitude in water's
    # k0 (Eq. attenuation_geom_reference), the dispersive k in the phase, A_abs = e^(-alpha d).
    # B and dT = T - d/c0 = (k/k0 - 1) d / c0 are interpolated linearly over the ray
    # triangles; for fields proportional to d (curvature 1/d across the fan) that error is below
    # (d dgamma^2 + ds^2 / d) / 8 times alpha0 in B and times (k - k0) / omega in dT.
    st = small_setup(N=16, n_rays=180)
    c, a0, ab = _homogeneous(st, 1.0)
    qx, qy = st.grid.mask_coords()
    pos = st.ring.positions()
    dg = math.pi / st.n_rays
    for f in (2e5, 7e5):
        om = 2 * math.pi * f
        tb, _ = step.tables_for(c, st, 1, absorption=ab, omega=om)
        G = green.build_green(tb, om, C0, Y)[0]
        k0, k, al = om / C0, lossy.wavenumber(om, C0, a0, Y), a0 * om ** Y
        for e in (0, 5, 11):
            v = tb.valid[e]
            d = np.hypot(qx - pos[e, 0], qy - pos[e, 1])[v]
            ref = (8 * math.pi * k0 * d) ** -0.5 * np.exp(1j * (k * d + math.pi / 4) - al * d)
            bound = (al + abs(k - k0)) * (d * dg * dg + st.ds ** 2 / d) / 8 + 1e-10
            assert np.all(np.abs(G[e][v] - ref) / np.abs(ref) <= bound)
        # at the receivers (chords)
        g = green.direct_data(tb, om, C0, Y)
        dr = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
        v = tb.rx_valid
        ref = (8 * math.pi * k0 * dr[v]) ** -0.5 * np.exp(1j * (k * dr[v] + math.pi / 4)
                                                          - al * dr[v])
        assert np.max(np.abs(g[v] - ref) / np.abs(ref)) < 1e-4


def test_linked_rays_carry_the_absorption_integral():
    # Linked rays in a homogeneous absorbing medium are chords: B = alpha0 |x_r - x_e|.
    ring = Ring(10, 0.02)
    nx = 111
    g = Grid(nx, nx, 0.4e-3, -(nx - 1) * 0.2e-3, -(nx - 1) * 0.2e-3, 0.018)
    a0 = ph.db_to_neper(1.0, Y)
    om = 2 * math.pi * 5e5
    al = np.full((nx, nx), a0)
    n_om = lossy.tracing_index(np.ones((nx, nx)), al, om, Y, C0)
    lk = link_receivers(n_om, g, ring, 40, 0.2e-3, 400, emitters=[0, 4], alpha=al)
    pos = ring.positions()
    for a, e in enumerate([0, 4]):
        for r in range(ring.n):
            if r != e:
                assert lk.valid[a, r]
                chord = math.hypot(*(pos[r] - pos[e]))
                assert abs(lk.B[a, r] - a0 * chord) <= 1e-8 * a0 * chord


def test_dispersion_cancelling_sound_speed_gives_straight_rays():
    # c0 / c = 1 - c0 tan(pi y/2) omega*^(y-1) alpha0 makes the traced map n_omega* = 1: at
    # omega* the rays are straight (T = d / c0) and B is the exact line integral of the linear
    # alpha0 = a + g . x (trapezoid rule and cubic B-spline are exact for linear functions);
    # at another frequency the map is not uniform and the rays bend.
    st = small_setup(N=8, n_rays=60)
    X, Yg = ph.node_coords(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0)
    a_c, gx, gy = ph.db_to_neper(0.5, Y), ph.db_to_neper(10.0, Y), ph.db_to_neper(-6.0, Y)
    alpha0 = a_c + gx * X + gy * Yg                           # per metre of position
    om_star = 2 * math.pi * 5e5
    kappa = C0 * lossy.tan_py(Y) * om_star ** (Y - 1.0)
    c = C0 / (1.0 - kappa * alpha0)
    ab = lossy.Absorption(alpha0, Y)
    pos = st.ring.positions()
    for om, straight in ((om_star, True), (4 * om_star, False)):
        n_om = lossy.tracing_index(C0 / c, alpha0, om, Y, C0)
        s = trace(n_om, st.grid, st.ring, st.n_rays, st.ds, st.max_steps, emitters=[1, 6],
                  alpha=ab.alpha0)
        p = pos[s.emitter]
        d = np.hypot(s.x - p[:, :1], s.y - p[:, 1:2])
        ok = np.isfinite(d)
        dev = np.max(np.abs(s.T[ok] * C0 - d[ok]))
        if straight:
            assert dev < 1e-12
            ux, uy = (s.x - p[:, :1]) / np.where(d > 0, d, 1), (s.y - p[:, 1:2]) / np.where(d > 0, d, 1)
            a_e = a_c + gx * p[:, :1] + gy * p[:, 1:2]
            exact = a_e * d + (gx * ux + gy * uy) * d * d / 2
            assert np.max(np.abs(s.B[ok] - exact[ok])) < 1e-12 * np.max(np.abs(exact[ok]))
        else:
            assert dev > 1e-7


def test_alpha0_zero_reproduces_the_lossless_step_bit_for_bit():
    st = small_setup(N=16, n_rays=90)
    c_true = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0,
                                   seed=6, amp=30.0, sigma=3e-3, centre_radius=4e-3,
                                   mask_radius=st.grid.mask_radius)
    om = [2 * math.pi * 250e3, 2 * math.pi * 400e3]
    dom = [2 * math.pi * 150e3] * 2
    data = step.synthesize(c_true, st, om, ph.complex_noise((2, 16, 16), 3), "smooth", 3)
    c = np.full_like(c_true, C0)
    zero = lossy.Absorption(np.zeros_like(c), Y)
    for w in (1, 3):
        a, pa = step.frequency_step(c_true * 0.999 + 1.5, st, om, dom, data, 0.12, window=w,
                                    return_parts=True)
        b, pb = step.frequency_step(c_true * 0.999 + 1.5, st, om, dom, data, 0.12, window=w,
                                    return_parts=True, absorption=zero)
        assert np.array_equal(a, b)
        assert np.array_equal(pa["dm"], pb["dm"])
        for fa, fb in zip(pa["freqs"], pb["freqs"]):
            for key in ("g", "R", "G", "H"):
                assert np.array_equal(fa[key], fb[key]), key
    d0 = step.synthesize(c_true, st, om, np.zeros((2, 16, 16)), "smooth", 3)
    d1 = step.synthesize(c_true, st, om, np.zeros((2, 16, 16)), "smooth", 3, absorption=zero)
    assert np.array_equal(d0, d1)
    assert c.shape == c_true.shape


def test_consistent_lossy_data_give_zero_update():
    st = small_setup(N=16, n_rays=90)
    c = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0,
                              seed=3, amp=20.0, sigma=4e-3, centre_radius=4e-3,
                              mask_radius=st.grid.mask_radius)
    a = ph.db_to_neper(ph.gaussian_absorption(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0,
                                              st.grid.y0, seed=3, sigma=4e-3,
                                              centre_radius=4e-3,
                                              mask_radius=st.grid.mask_radius), Y)
    ab = lossy.Absorption(a, Y)
    om = [2 * math.pi * 200e3, 2 * math.pi * 320e3]
    data = step.synthesize(c, st, om, np.zeros((2, 16, 16)), "smooth", 1, noise_level=0.0,
                           absorption=ab)
    c1, parts = step.frequency_step(c, st, om, om, data, 0.12, absorption=ab, return_parts=True)
    assert all(np.all(f["R"] == 0) for f in parts["freqs"])
    assert np.all(parts["dm"] == 0)
    # the rays of the two frequencies differ (dispersion), so the tables were traced twice
    t0, t1 = parts["freqs"][0]["tables"], parts["freqs"][1]["tables"]
    v = t0.valid & t1.valid
    assert np.max(np.abs(t0.T[v] - t1.T[v])) > 1e-10
    assert np.max(np.abs(c1 - c) / c) < 4e-16


def test_absorbing_blob_delays_amplitude_and_advances_phase():
    # An alpha0 blob inside water (c = c0): k < k0 in the blob (tan(pi y/2) < 0) so nodes
    # behind it are reached earlier, more so at the higher frequency, and with less amplitude.
    st = small_setup(N=16, n_rays=180)
    c = np.full((st.grid.ny, st.grid.nx), C0)
    X, Yg = ph.node_coords(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0)
    a = ph.db_to_neper(1.0 * np.exp(-(X ** 2 + Yg ** 2) / (2 * 3e-3 ** 2)), Y)
    ab = lossy.Absorption(a, Y)
    tw, _ = step.tables_for(c, st, 1)
    lo, _ = step.tables_for(c, st, 1, absorption=ab, omega=2 * math.pi * 2e5)
    hi, _ = step.tables_for(c, st, 1, absorption=ab, omega=2 * math.pi * 8e5)
    e = 0
    qx, qy = st.grid.mask_coords()
    pos = st.ring.positions()[e]
    behind = (qx < -8e-3) & (np.abs(qy) < 1e-3) & tw.valid[e] & lo.valid[e] & hi.valid[e]
    assert np.abs(pos[1]) < 1e-12 and pos[0] > 0 and behind.sum() > 3
    assert np.all(hi.T[e][behind] < lo.T[e][behind])
    assert np.all(lo.T[e][behind] < tw.T[e][behind])
    assert np.all(hi.B[e][behind] > 0) and np.allclose(hi.B[e][behind], lo.B[e][behind],
                                                       rtol=0.05)


@pytest.fixture(scope="module")
def lossy_psf():
    # Homogeneous absorbing medium (c = c0, alpha0 = 5 dB MHz^-y cm^-1 everywhere, exaggerated
    # so that the absorption over the ring is large: exp(-2 alpha R) ~ 0.4), ring of 128 at
    # R = 25 mm, 300 kHz: one back-projection of one point scatterer's Born data.
    from tests.oracle_fixtures import small_setup as ss

    st = ss(N=128, R=0.025, dx=0.25e-3, n_rays=360)
    c, a0, ab = _homogeneous(st, 5.0)
    om = 2 * math.pi * 300e3
    tb, _ = step.tables_for(c, st, 1, absorption=ab, omega=om)
    G, H, Hx, Hy = green.build_green(tb, om, C0, Y)
    qx, qy = st.grid.mask_coords()
    p0 = int(np.argmin((qx - 3e-3) ** 2 + (qy + 2e-3) ** 2))
    dm0 = 1e-9
    delta = np.zeros(qx.size)
    delta[p0] = dm0
    w = step.born_weight(c, st, om, ab)
    N = st.ring.n
    R = -born.forward(G, w, delta) * ~np.eye(N, dtype=bool)
    cq = np.full(qx.size, C0)
    S = born.backproject_weight(om, om, cq, np.full(qx.size, a0), Y)
    tw, _ = step.tables_for(c, st, 1)
    _, Hw, Hxw, Hyw = green.build_green(tw, om, C0)
    return dict(st=st, om=om, a0=a0, qx=qx, qy=qy, p0=p0, dm0=dm0, R=R, H=H, Hx=Hx, Hy=Hy,
                S=S, Hw=Hw, Hxw=Hxw, Hyw=Hyw, Sw=born.backproject_weight(om, om, cq))


def test_lossy_point_spread_function_of_one_step(lossy_psf):
    # Appendix D with Szabo's k: the kernel (1/2 pi) 2 k dk [J0^2 - J1^2](k |x - x0|) with the
    # dispersive k and dk = Domega dk/domega; at x0 the reciprocal Green's functions undo the
    # absorption exactly and S Upsilon_m is real, so the peak is exact up to the quadrature of
    # the angular weights (as in water).
    c = lossy_psf
    om, a0 = c["om"], c["a0"]
    k = lossy.wavenumber(om, C0, a0, Y)
    dk = om * lossy.dk_domega(om, C0, a0, Y)
    dm = born.backproject(c["R"], c["H"], c["Hx"], c["Hy"], c["S"])
    xd = np.hypot(c["qx"] - c["qx"][c["p0"]], c["qy"] - c["qy"][c["p0"]])
    h2 = c["st"].grid.dx ** 2
    psf = h2 * c["dm0"] * (2 * k * dk / (2 * math.pi)) * (j0(k * xd) ** 2 - j1(k * xd) ** 2)
    assert abs(dm[c["p0"]] / psf[c["p0"]] - 1) < 0.02
    lam = 2 * math.pi / k
    for rad in (0.5 * lam, lam):
        sel = xd < rad
        assert np.corrcoef(dm[sel], psf[sel])[0, 1] > 0.995
    # the lossless operator on the same data misses the peak by the uncompensated absorption
    dmw = born.backproject(c["R"], c["Hw"], c["Hxw"], c["Hyw"], c["Sw"])
    assert dmw[c["p0"]] / psf[c["p0"]] < 0.8
