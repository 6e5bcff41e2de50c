"""Least-squares fits of the polynomial arctangents used by the binning kernels.

The ray direction stored in the 16-bit step's compact records and the straight-ray guess of
the binning walk take the polar angle of a vector by octant reduction (t = min/max of |x|, |y|
in [0, 1]) and an odd polynomial t p(t^2) ~ atan(t). The coefficients are the least-squares fit
of atan on 2000 Chebyshev nodes of [0, 1] (absolute error), rounded to float:

  * 8 terms (degree 15), the record's ray angle: max error 4.1e-8 rad in exact arithmetic,
    below 3e-7 rad evaluated in FP32 as the kernel does;
  * 4 terms (degree 7), the walk's guess: max error 8.8e-5 rad (below 1e-4 rad).

Run as a script to print the coefficients in the order the kernels' Horner schemes take them
(highest power first).
"""
from __future__ import annotations

import numpy as np

N_NODES = 2000


def fit(n_terms: int, n_nodes: int = N_NODES) -> np.ndarray:
    """Coefficients c_k of sum_k c_k t^(2k+1) ~ atan(t) on [0, 1], lowest power first (FP64)."""
    t = 0.5 + 0.5 * np.cos(np.pi * (np.arange(n_nodes) + 0.5) / n_nodes)
    V = np.stack([t ** (2 * k + 1) for k in range(n_terms)], axis=1)
    return np.linalg.lstsq(V, np.arctan(t), rcond=None)[0]


def as_float(c: np.ndarray) -> list:
    """The coefficients as the kernels store them (FP32), lowest power first."""
    return [float(np.float32(x)) for x in c]


if __name__ == "__main__":
    for n in (8, 4):
        cf = as_float(fit(n))
        print(f"{n} terms, highest power first:", ", ".join(f"{x:.8g}f" for x in cf[::-1]))
