"""Pins of the oracle's frequency step (Section 3.4 update, Eq. residual, Section 6.3.2)."""
import math

import numpy as np

import phantoms as ph
from oracle import step
from oracle.medium import box_smooth
from tests.oracle_fixtures import C0, small_setup


def test_consistent_data_give_zero_update():
    # Data equal to the prediction of the current model: g_res = 0, so dm = 0 and c is
    # returned unchanged (up to the rounding of c -> m -> c).
    st = small_setup(N=16, n_rays=90)
    c = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0,
                              seed=3, amp=20.0, sigma=4e-3, centre_radius=4e-3,
                              mask_radius=st.grid.mask_radius)
    om = [2 * math.pi * 200e3]
    tb, ns = step.tables_for(c, st, 1)
    g, _ = step.predicted(tb, c, ns, st, om[0])
    c1, parts = step.frequency_step(c, st, om, om, g[None], 0.12, return_parts=True)
    assert np.all(parts["freqs"][0]["R"] == 0)
    assert np.all(parts["dm"] == 0)
    assert np.max(np.abs(c1 - c) / c) < 4e-16


def test_ray_born_and_ray_only_agree_without_smoothing():
    st = small_setup(N=16, n_rays=90)
    c = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0,
                              seed=4, amp=30.0, sigma=4e-3, centre_radius=4e-3,
                              mask_radius=st.grid.mask_radius)
    tb, ns = step.tables_for(c, st, 1)
    a, _ = step.predicted(tb, c, ns, st, 2 * math.pi * 300e3, "ray_born")
    b, _ = step.predicted(tb, c, ns, st, 2 * math.pi * 300e3, "ray_only")
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b))


def test_rough_part_enters_through_born_term():
    # With smoothing, g(m) = g_ray(m_s) + F[m_s](m - m_s) with m_s = (n_s / c0)^2.
    st = small_setup(N=16, n_rays=90)
    c = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0, st.grid.y0,
                              seed=4, amp=30.0, sigma=2e-3, centre_radius=4e-3,
                              mask_radius=st.grid.mask_radius)
    tb, ns = step.tables_for(c, st, 5)
    assert np.allclose(ns, box_smooth(C0 / c, 5))
    a, _ = step.predicted(tb, c, ns, st, 2 * math.pi * 300e3, "ray_born")
    b, _ = step.predicted(tb, c, ns, st, 2 * math.pi * 300e3, "ray_only")
    assert np.max(np.abs(a - b)) > 1e-5 * np.max(np.abs(b))


def test_update_is_linear_in_step_length_and_frequency_spacing():
    st = small_setup(N=16, n_rays=90)
    c_true = ph.gaussian_inclusion(st.grid.nx, st.grid.ny, st.grid.dx, st.grid.x0,
                                   st.grid.y0, seed=6, amp=30.0, sigma=3e-3,
                                   centre_radius=4e-3, mask_radius=st.grid.mask_radius)
    om = [2 * math.pi * 250e3]
    noise = np.zeros((1, 16, 16), dtype=complex)
    data = step.synthesize(c_true, st, om, noise)
    c = np.full_like(c_true, C0)
    q = st.grid.mask_index()
    _, p1 = step.frequency_step(c, st, om, om, data, 0.12, return_parts=True)
    _, p2 = step.frequency_step(c, st, om, [2 * om[0]], data, 0.12, return_parts=True)
    assert np.allclose(p2["dm"], 2 * p1["dm"], rtol=1e-12, atol=0)
    c1 = step.update(c, p1["dm"], 0.12, st.grid)
    m1 = 1.0 / c1.ravel()[q] ** 2
    assert np.allclose(m1, 1 / C0 ** 2 + 0.12 * p1["dm"], rtol=1e-14, atol=0)
    outside = np.setdiff1d(np.arange(c.size), q)
    assert np.all(c1.ravel()[outside] == C0)
    # the step moves the model towards the (faster) inclusion: dc correlates positively
    dc = (c1 - C0).ravel()[q]
    assert np.corrcoef(dc, (c_true - C0).ravel()[q])[0, 1] > 0


def test_residual_masks_diagonal_and_invalid_pairs():
    g = np.ones((4, 4), dtype=complex)
    data = np.zeros((4, 4), dtype=complex)
    valid = np.ones((4, 4), dtype=bool)
    valid[1, 2] = False
    R = step.residual(g, data, valid)
    assert np.all(np.diag(R) == 0) and R[1, 2] == 0 and R[2, 1] == 1


def test_tables_in_worker_processes_are_the_same():
    # the process-parallel table builder stacks the rows of transducer chunks: identical
    # tables to the one-process build
    from oracle import step as ostep
    from tests.oracle_fixtures import small_setup
    import phantoms as ph

    st = small_setup(N=12, R=0.012, dx=0.5e-3, n_rays=60)
    g = st.grid
    c = ph.gaussian_inclusion(g.nx, g.ny, g.dx, g.x0, g.y0, seed=4, amp=30.0, sigma=2e-3,
                              centre_radius=3e-3, mask_radius=g.mask_radius)
    a, _ = ostep.tables_for(c, st, 3)
    b, _ = ostep.tables_for(c, st, 3, workers=3)
    for f in ("valid", "T", "A", "ux", "uy", "K", "rx_valid", "rx_T", "rx_A", "rx_K"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_fp32_map_option_rounds_only_the_map():
    # map32 changes nothing but the map's representation: in water (exact in FP32) the tables
    # are identical; in a heterogeneous medium they differ at the rounding level only
    from oracle import step as ostep
    from tests.oracle_fixtures import small_setup
    import phantoms as ph

    st = small_setup(N=12, R=0.012, dx=0.5e-3, n_rays=60)
    g = st.grid
    cw = np.full((g.ny, g.nx), C0)
    a, _ = ostep.tables_for(cw, st, 1)
    b, _ = ostep.tables_for(cw, st, 1, map32=True)
    assert np.array_equal(a.T, b.T) and np.array_equal(a.A, b.A)
    c = ph.gaussian_inclusion(g.nx, g.ny, g.dx, g.x0, g.y0, seed=4, amp=30.0, sigma=2e-3,
                              centre_radius=3e-3, mask_radius=g.mask_radius)
    a, ns = ostep.tables_for(c, st, 3)
    b, ns32 = ostep.tables_for(c, st, 3, map32=True)
    assert np.array_equal(ns32, ns.astype(np.float32).astype(np.float64))
    v = a.valid & b.valid
    assert np.max(np.abs(a.T[v] - b.T[v]) / a.T[v]) < 1e-6
