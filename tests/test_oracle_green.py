"""Pins of the oracle's Green's functions and angular weights (Eqs. 2D_greens,
greens-time-reversed, Appendix B, Section 3.4)."""
import math

import numpy as np
from scipy.special import hankel1

from oracle import green
from tests.oracle_fixtures import C0, water_tables


def test_water_green_matches_appendix_b_closed_form():
    st, tb = water_tables()
    qx, qy = st.grid.mask_coords()
    pos = st.ring.positions()
    for f in (150e3, 600e3):
        om = 2 * math.pi * f
        k0 = om / C0
        G, H, Hx, Hy = green.build_green(tb, om)
        for e in (0, 7, 31):
            d = np.hypot(qx - pos[e, 0], qy - pos[e, 1])
            v = tb.valid[e]
            g0 = (8 * math.pi * k0 * d) ** -0.5 * np.exp(1j * (k0 * d + math.pi / 4))
            assert np.max(np.abs(G[e][v] - g0[v]) / np.abs(g0[v])) < 1e-10
            assert np.all(G[e][~v] == 0) and np.all(H[e][~v] == 0)


def test_water_green_is_the_hankel_asymptote():
    # g0 is the large-k0 r asymptote of the exact 2D Green's function (i/4) H0^(1)(k0 r);
    # relative error of that expansion ~ 1/(8 k0 r).
    st, tb = water_tables()
    qx, qy = st.grid.mask_coords()
    pos = st.ring.positions()
    om = 2 * math.pi * 500e3
    k0 = om / C0
    G = green.build_green(tb, om)[0]
    e = 4
    d = np.hypot(qx - pos[e, 0], qy - pos[e, 1])
    sel = tb.valid[e] & (k0 * d >= 10)
    exact = 0.25j * hankel1(0, k0 * d[sel])
    rel = np.abs(G[e][sel] - exact) / np.abs(exact)
    assert np.all(rel <= 1.1 / (8 * k0 * d[sel]))


def test_reciprocal_green_inverts_amplitude_and_phase():
    # Eq. greens-time-reversed: g_dagger g = 1 where the table is valid.
    st, tb = water_tables()
    om = 2 * math.pi * 400e3
    G, H, Hx, Hy = green.build_green(tb, om)
    a = green.angular_weights(tb)
    v = tb.valid & (a > 0)
    assert np.max(np.abs(H[v] / a[v] * G[v] - 1.0)) < 1e-12
    assert np.allclose(Hx[v], H[v] * tb.ux[v]) and np.allclose(Hy[v], H[v] * tb.uy[v])


def test_angular_weights_water_closed_form():
    # In water gamma(x, e) is the angle of x - x_e, so |dgamma/dpsi| = R (R - x.nu_e)/|x-x_e|^2
    # with nu_e the outward normal; the central difference approximates it to
    # O((dpsi R / d)^2) (leading constant 1/3 on the normal; up to 1 off it).
    st, tb = water_tables()
    N, R = st.ring.n, st.ring.radius
    a = green.angular_weights(tb)
    qx, qy = st.grid.mask_coords()
    psi = st.ring.angles()
    dpsi = 2 * math.pi / N
    for e in (0, 9, 20):
        nu = np.array([math.cos(psi[e]), math.sin(psi[e])])
        xe = R * nu
        d = np.hypot(qx - xe[0], qy - xe[1])
        exact = dpsi * R * (R - (qx * nu[0] + qy * nu[1])) / d ** 2
        v = tb.valid[e]
        rel = np.abs(a[e][v] - exact[v]) / exact[v]
        bound = (dpsi * R / d[v]) ** 2 + 5e-3
        assert np.all(rel < bound), np.max(rel / bound)


def test_angular_weights_sum_to_two_pi():
    # Central differences of a monotone angle telescope: sum_e a_e(x) = 2 pi inside the ring.
    st, tb = water_tables()
    a = green.angular_weights(tb)
    full = tb.valid.all(axis=0)
    assert np.max(np.abs(a[:, full].sum(axis=0) - 2 * math.pi)) < 1e-12


def test_phase_reduction():
    T = np.array([1e-4, 2.5e-5])
    K = np.array([0, 1])
    om = 2 * math.pi * 1.2e6
    ph = green.phase(T, K, om)
    assert np.all((ph >= 0) & (ph < 2 * math.pi))
    ref = np.angle(np.exp(1j * (om * T + math.pi / 4 - K * math.pi / 2))) % (2 * math.pi)
    assert np.allclose(ph, ref, atol=1e-9)
    assert np.allclose(green.wrap(np.array([0.0, math.pi, -math.pi, 1.5 * math.pi])),
                       [0.0, math.pi, math.pi, -0.5 * math.pi])


def _receiver_distances(st):
    pos = st.ring.positions()
    return np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])


def test_direct_data_water_matches_appendix_b_at_the_receivers():
    # App. B: in water g(omega, r, e) = [8 pi k0 |x_r - x_e|]^-1/2 exp(i (k0 |x_r - x_e| + pi/4))
    # for every pair the fan brackets; the other pairs are zero.
    st, tb = water_tables()
    d = _receiver_distances(st)
    N = st.ring.n
    assert tb.rx_valid[~np.eye(N, dtype=bool)].mean() > 0.9
    for f in (150e3, 600e3):
        om = 2 * math.pi * f
        k0 = om / C0
        g = green.direct_data(tb, om)
        v = tb.rx_valid
        g0 = (8 * math.pi * k0 * d[v]) ** -0.5 * np.exp(1j * (k0 * d[v] + math.pi / 4))
        assert np.max(np.abs(g[v] - g0) / np.abs(g0)) < 1e-10
        assert np.all(g[~v] == 0)


def test_direct_data_is_the_hankel_asymptote_at_the_receivers():
    # The receiver values approach the exact 2D Green's function (i/4) H0^(1)(k0 r) (SciPy) with
    # the asymptotic error 1/(8 k0 r): independent of the closed form's own phase and amplitude.
    st, tb = water_tables()
    d = _receiver_distances(st)
    om = 2 * math.pi * 500e3
    k0 = om / C0
    g = green.direct_data(tb, om)
    v = tb.rx_valid & (k0 * d >= 10)
    assert v.sum() > 500
    exact = 0.25j * hankel1(0, k0 * d[v])
    rel = np.abs(g[v] - exact) / np.abs(exact)
    assert np.all(rel <= 1.1 / (8 * k0 * d[v]))


def test_direct_data_caustic_shift():
    # Eq. phase-discretised: each caustic the ray has passed retards the phase by pi/2, so a
    # table with K = 1 gives -i times, and K = 2 gives -1 times, the K = 0 value.
    import dataclasses

    st, tb = water_tables()
    om = 2 * math.pi * 300e3
    g0 = green.direct_data(tb, om)
    for K, factor in ((1, -1j), (2, -1.0), (3, 1j), (4, 1.0)):
        tk = dataclasses.replace(tb, rx_K=np.full_like(tb.rx_K, K))
        gk = green.direct_data(tk, om)
        v = tb.rx_valid
        assert np.max(np.abs(gk[v] - factor * g0[v])) < 1e-12 * np.max(np.abs(g0[v]))


def test_synthesized_noise_level():
    # O11: sigma = 1 % of the rms of the clean data over the valid pairs with e != r; the
    # measured noise rms over those pairs agrees within its seeded sampling error.
    import phantoms as ph
    from oracle import step as ostep

    st, tb = water_tables()
    N = st.ring.n
    c = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0,
                              seed=3, amp=20.0, sigma=3e-3, centre_radius=4e-3,
                              mask_radius=st.grid.mask_radius)
    oms = [2 * math.pi * 250e3, 2 * math.pi * 400e3]
    clean = ostep.synthesize(c, st, oms, np.zeros((2, N, N)))
    noisy = ostep.synthesize(c, st, oms, ph.complex_noise((2, N, N), 7))
    keep = tb.rx_valid & ~np.eye(N, dtype=bool)
    for k in range(2):
        rms = math.sqrt(np.mean(np.abs(clean[k][keep]) ** 2))
        sigma = math.sqrt(np.mean(np.abs(noisy[k][keep] - clean[k][keep]) ** 2))
        n = int(keep.sum())
        # the rms of n unit complex Gaussians has relative standard deviation ~ 1/(2 sqrt(n))
        assert abs(sigma / (0.01 * rms) - 1.0) < 4.0 / (2.0 * math.sqrt(n))
        # and the noise is the only difference
        diff = noisy[k] - clean[k] - 0.01 * rms * ph.complex_noise((2, N, N), 7)[k]
        assert np.max(np.abs(diff)) < 1e-15 * rms
