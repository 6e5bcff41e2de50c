"""Pins of the oracle's grid-to-ray interpolation and smoothing (Section 4.5, Section 6.3.2)."""
import numpy as np
import pytest
from scipy.ndimage import uniform_filter

from oracle.medium import Grid, Ring, box_smooth, bspline


def _grid(n=24, dx=0.5e-3):
    x0 = -(n - 1) * dx / 2
    return Grid(n, n, dx, x0, x0, 0.9 * abs(x0))


def _points(g, m=200, seed=0):
    rng = np.random.default_rng(seed)
    lo, hi = g.x0 + 3 * g.dx, g.x0 + (g.nx - 4) * g.dx
    return rng.uniform(lo, hi, m), rng.uniform(lo, hi, m)


def test_bspline_reproduces_linear_maps():
    # A uniform cubic B-spline reproduces polynomials of degree <= 1 exactly.
    g = _grid()
    X, Y = g.coords()
    f = 1.02 + 3.0 * X - 7.0 * Y
    x, y = _points(g)
    v, gx, gy, hxx, hxy, hyy = bspline(f, g, x, y)
    assert np.max(np.abs(v - (1.02 + 3.0 * x - 7.0 * y))) < 1e-13
    assert np.max(np.abs(gx - 3.0)) < 1e-9 and np.max(np.abs(gy + 7.0)) < 1e-9
    assert max(np.max(np.abs(h)) for h in (hxx, hxy, hyy)) < 1e-4


def test_bspline_quadratic_shift():
    # Closed form: the approximating cubic B-spline of samples of u^2 is u^2 + 1/3
    # (index units), so f = x^2 gives x^2 + dx^2/3, gradient 2x and second derivative 2.
    g = _grid()
    X, Y = g.coords()
    f = X ** 2 + 2 * Y ** 2
    x, y = _points(g, seed=1)
    v, gx, gy, hxx, hxy, hyy = bspline(f, g, x, y)
    exact = x ** 2 + 2 * y ** 2 + 3 * g.dx ** 2 / 3.0
    assert np.max(np.abs(v - exact)) < 1e-15
    assert np.max(np.abs(gx - 2 * x)) < 1e-11 and np.max(np.abs(gy - 4 * y)) < 1e-11
    assert np.max(np.abs(hxx - 2)) < 1e-6 and np.max(np.abs(hyy - 4)) < 1e-6
    assert np.max(np.abs(hxy)) < 1e-6


def test_bspline_derivatives_match_finite_differences():
    g = _grid()
    rng = np.random.default_rng(3)
    f = 1.0 + 0.05 * rng.standard_normal((g.ny, g.nx))
    x, y = _points(g, seed=2)
    e = 1e-7
    v, gx, gy, hxx, hxy, hyy = bspline(f, g, x, y)
    vxp = bspline(f, g, x + e, y)
    vxm = bspline(f, g, x - e, y)
    vyp = bspline(f, g, x, y + e)
    vym = bspline(f, g, x, y - e)
    scale_g = np.max(np.abs(gx)) + np.max(np.abs(gy))
    assert np.max(np.abs((vxp[0] - vxm[0]) / (2 * e) - gx)) < 1e-5 * scale_g
    assert np.max(np.abs((vyp[0] - vym[0]) / (2 * e) - gy)) < 1e-5 * scale_g
    scale_h = np.max(np.abs(hxx)) + np.max(np.abs(hyy))
    assert np.max(np.abs((vxp[1] - vxm[1]) / (2 * e) - hxx)) < 1e-5 * scale_h
    assert np.max(np.abs((vyp[2] - vym[2]) / (2 * e) - hyy)) < 1e-5 * scale_h
    assert np.max(np.abs((vyp[1] - vym[1]) / (2 * e) - hxy)) < 1e-5 * scale_h


def test_bspline_constant_map_has_zero_gradient_everywhere():
    g = _grid()
    f = np.full((g.ny, g.nx), 1.0)
    x = np.linspace(g.x0 - g.dx, g.x0 + g.nx * g.dx, 101)
    v, gx, gy, hxx, hxy, hyy = bspline(f, g, x, 0.3 * x)
    assert np.all(v == 1.0) or np.max(np.abs(v - 1.0)) < 1e-15
    assert max(np.max(np.abs(a)) for a in (gx, gy, hxx, hxy, hyy)) < 1e-9


@pytest.mark.parametrize("w", [1, 3, 7, 13])
def test_box_smooth_matches_library_moving_average(w):
    rng = np.random.default_rng(w)
    f = rng.standard_normal((37, 41))
    ref = uniform_filter(f, size=w, mode="nearest")
    assert np.max(np.abs(box_smooth(f, w) - ref)) < 1e-13


def test_box_smooth_rejects_even_window():
    with pytest.raises(ValueError):
        box_smooth(np.ones((5, 5)), 4)


def test_ring_positions():
    r = Ring(8, 0.05, psi0=0.1)
    p = r.positions()
    assert np.allclose(np.hypot(p[:, 0], p[:, 1]), 0.05, rtol=0, atol=1e-17)
    assert np.isclose(np.arctan2(p[0, 1], p[0, 0]), 0.1)
