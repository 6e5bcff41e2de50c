"""The polynomial arctangents of the binning kernels: their coefficients are the documented
least-squares fit (paper_2211_00316_amd/fit_atan.py), and, evaluated in FP32 the way the
kernels evaluate them, they meet the stated bounds over every direction. The ray angle feeds
the angular Jacobian factors |d gamma_e / d e| De of Eq. sound_speed_update2 (Section 3.4)."""
import math
import os
import re

import numpy as np

from paper_2211_00316_amd import fit_atan

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2211_00316_amd", "csrc", "rb_trace.hip")


def _function_body(name):
    s = open(SRC).read()
    i = s.index(f"float {name}(float y, float x)")
    return s[i:s.index("\n}\n", i)]


def _coefficients(name):
    """The literals of the Horner scheme, highest power first."""
    body = _function_body(name)
    body = body[body.index("t2 = t * t;"):body.index("if (ay > ax)")]
    return [float(x) for x in re.findall(r"-?\d+\.\d+(?:e-?\d+)?(?=f)", body)]


def _fma32(a, b, c):
    # a b is exact in FP64 for FP32 operands; one rounding of the sum to FP32 as fmaf does
    # (up to rare double rounding, far below the bounds checked here)
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def _atan2_fp32(y, x, coef_high_first):
    y = y.astype(np.float32)
    x = x.astype(np.float32)
    ax, ay = np.abs(x), np.abs(y)
    t = (np.minimum(ax, ay) / np.maximum(np.maximum(ax, ay), np.float32(1e-30))).astype(np.float32)
    t2 = (t * t).astype(np.float32)
    p = np.full_like(t, np.float32(coef_high_first[0]))
    for c in coef_high_first[1:]:
        p = _fma32(p, t2, np.float32(c))
    a = (t * p).astype(np.float32)
    a = np.where(ay > ax, np.float32(1.57079633) - a, a)
    a = np.where(x < 0, np.float32(3.14159265) - a, a)
    return np.where(y < 0, -a, a).astype(np.float32)


def test_coefficients_are_the_documented_fit():
    for name, n in (("ray_atan2", 8), ("guess_atan2", 4)):
        want = fit_atan.as_float(fit_atan.fit(n))[::-1]
        got = _coefficients(name)
        assert len(got) == n, (name, got)
        assert np.allclose(got, want, rtol=2e-7, atol=0), (name, got, want)


def test_fit_bounds_in_exact_arithmetic():
    t = np.linspace(0.0, 1.0, 200001)
    for n, bound in ((8, 5e-8), (4, 1e-4)):
        c = fit_atan.fit(n)
        p = sum(ck * t ** (2 * k + 1) for k, ck in enumerate(c))
        assert np.max(np.abs(p - np.arctan(t))) < bound


def test_fp32_evaluation_bounds_over_all_directions():
    ang = np.linspace(-math.pi, math.pi, 400001)
    rng = np.random.Generator(np.random.PCG64(11))
    r = np.exp(rng.uniform(-8, 8, ang.size))   # scale independence over many magnitudes
    x, y = r * np.cos(ang), r * np.sin(ang)
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    exact = np.arctan2(y32.astype(np.float64), x32.astype(np.float64))
    for name, bound in (("ray_atan2", 3e-7), ("guess_atan2", 1e-4)):
        got = _atan2_fp32(y32, x32, _coefficients(name)).astype(np.float64)
        err = np.abs(np.angle(np.exp(1j * (got - exact))))
        assert np.max(err) < bound, (name, np.max(err))
