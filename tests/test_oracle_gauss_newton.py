"""Pins of the Gauss-Newton and prototype Born oracles (Section 6.3.2 b and c; Eqs.
linearised-linearised-subproblem, hessian-action, functional-gradient with Q = 1):
conjugate gradients against a direct solve, the Hessian action against the dense Jacobian
built from the brute-force Born sum, the step against the least-squares solution, the
first iterate against the exact line search, and exact recovery of noise-free linear data."""
import math

import numpy as np

import phantoms as ph
from oracle import born, gauss_newton as gn, green, step as ostep
from tests.oracle_fixtures import C0, small_setup


def _tiny():
    # 16 transducers on a 6 mm ring, coarse grid: a few dozen mask nodes, 240 kept pairs
    st = small_setup(N=16, R=0.006, dx=0.9e-3, n_rays=90)
    return st


def test_cg_matches_a_direct_solve():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((30, 30))
    A = M @ M.T + 0.5 * np.eye(30)
    b = rng.standard_normal(30)
    # n iterations in exact arithmetic; twice that in floating point (lost orthogonality)
    x, hist = gn.cg(lambda v: A @ v, b, 60)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(x)
    # the A-norm of the error decreases at every iterate
    xs = np.linalg.solve(A, b)
    errs = []
    for k in range(1, 12):
        xk, _ = gn.cg(lambda v: A @ v, b, k)
        errs.append(float((xk - xs) @ A @ (xk - xs)))
    assert all(b2 < a2 for a2, b2 in zip(errs, errs[1:]))


def _dense_jacobian(G, w, keep):
    """Columns J[:, p] = J e_p from the brute-force triple sum, as a complex matrix."""
    N, P = G.shape
    cols = []
    for p in range(P):
        v = np.zeros(P)
        v[p] = w[p]
        cols.append(np.where(keep, born.forward_bruteforce(G, v), 0.0).ravel())
    return np.stack(cols, axis=1)


def test_hessian_action_equals_dense_jacobian_normal_matrix():
    st = _tiny()
    tb = gn.water_tables(st)
    N = st.ring.n
    keep = tb.rx_valid & ~np.eye(N, dtype=bool)
    oms = [2 * math.pi * 250e3, 2 * math.pi * 300e3]
    ops = []
    Hd = 0
    for om in oms:
        G = green.build_green(tb, om)[0]
        w = np.full(G.shape[1], om ** 2 * st.grid.dx ** 2)
        ops.append((G, w, keep))
        J = _dense_jacobian(G, w, keep)
        Hd = Hd + np.real(J.conj().T @ J)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(Hd.shape[0])
    y = rng.standard_normal(Hd.shape[0])
    Hx = gn.normal_apply(ops, x)
    assert np.linalg.norm(Hx - Hd @ x) <= 1e-11 * np.linalg.norm(Hd @ x)
    # symmetric, positive semi-definite
    assert abs(y @ gn.normal_apply(ops, x) - x @ gn.normal_apply(ops, y)) <= 1e-11 * abs(y @ Hx)
    assert x @ Hx > 0


def _linear_problem(seed=3):
    st = _tiny()
    g = st.grid
    c_true = ph.gaussian_inclusion(g.nx, g.ny, g.dx, g.x0, g.y0, seed=seed, amp=25.0,
                                   sigma=1.5e-3, centre_radius=1.5e-3, mask_radius=g.mask_radius)
    oms = [2 * math.pi * 250e3, 2 * math.pi * 300e3]
    N = st.ring.n
    data = ostep.synthesize(c_true, st, oms, np.zeros((2, N, N)), background="water")
    return st, c_true, oms, data


def test_gauss_newton_step_is_the_least_squares_solution():
    # full CG (as many iterations as unknowns) reaches the minimiser of the linearised
    # objective: the least-squares solution of the stacked real system [Re J; Im J] x = -[Re R; Im R]
    st, c_true, oms, data = _linear_problem()
    c = np.full_like(c_true, C0)
    P = st.grid.mask_index().size
    _, parts = gn.gauss_newton_step(c, st, oms, data, 1.0, 10 * P, model="water",
                                    return_parts=True)
    A, rhs = [], []
    for (G, w, keep), R in zip(parts["ops"], parts["residuals"]):
        J = _dense_jacobian(G, w, keep)
        A += [J.real, J.imag]
        rhs += [-R.ravel().real, -R.ravel().imag]
    xs = np.linalg.lstsq(np.vstack(A), np.concatenate(rhs), rcond=None)[0]
    assert np.linalg.norm(parts["dm"] - xs) <= 1e-6 * np.linalg.norm(xs)


def test_first_cg_iterate_is_the_exact_line_search_along_the_gradient():
    st, c_true, oms, data = _linear_problem()
    c = np.full_like(c_true, C0)
    _, parts = gn.gauss_newton_step(c, st, oms, data, 1.0, 1, model="water", return_parts=True)
    g = parts["grad"]
    Hg = gn.normal_apply(parts["ops"], g)
    x1 = -(g @ g) / (g @ Hg) * g
    assert np.linalg.norm(parts["dm"] - x1) <= 1e-12 * np.linalg.norm(x1)


def test_prototype_born_recovers_noise_free_linear_data():
    # Born data about water are linear in m: the full Gauss-Newton step from water returns
    # the true perturbation where the kept pairs determine it (full column rank here)
    st, c_true, oms, data = _linear_problem()
    q = st.grid.mask_index()
    c = np.full_like(c_true, C0)
    c_new = gn.gauss_newton_step(c, st, oms, data, 1.0, 10 * q.size, model="water")
    dm_true = 1.0 / c_true.ravel()[q] ** 2 - 1.0 / C0 ** 2
    dm = 1.0 / c_new.ravel()[q] ** 2 - 1.0 / C0 ** 2
    assert np.linalg.norm(dm - dm_true) <= 1e-6 * np.linalg.norm(dm_true)


def test_ray_model_in_water_is_the_prototype():
    # in water the traced tables are the analytic ones (to rounding), so the two models take
    # the same step
    st, c_true, oms, data = _linear_problem()
    c = np.full_like(c_true, C0)
    q = st.grid.mask_index()
    a = gn.gauss_newton_step(c, st, oms, data, 1.0, 8, model="water")
    b = gn.gauss_newton_step(c, st, oms, data, 1.0, 8, model="ray")
    da, db = (a - C0).ravel()[q], (b - C0).ravel()[q]
    assert np.linalg.norm(da - db) <= 1e-7 * np.linalg.norm(da)


def test_water_tables_are_the_traced_ones_in_water():
    st = _tiny()
    c = np.full((st.grid.ny, st.grid.nx), C0)
    tr, _ = ostep.tables_for(c, st, 1)
    wt = gn.water_tables(st)
    v = tr.valid
    assert np.max(np.abs(tr.T[v] - wt.T[v]) / wt.T[v]) < 1e-12
    assert np.max(np.abs(tr.A[v] - wt.A[v]) / wt.A[v]) < 1e-10
    assert np.array_equal(tr.rx_valid, tr.rx_valid & wt.rx_valid)
