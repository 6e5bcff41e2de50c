"""Small shared setups for the oracle pins (water ring, fine grid)."""
import functools
import math

import numpy as np

from oracle.medium import Grid, Ring
from oracle.step import StepSetup

C0 = 1500.0


def small_setup(N=32, R=0.02, dx=0.4e-3, n_rays=180, ds=0.2e-3, margin=2e-3):
    nx = int(math.ceil(2 * (R + margin) / dx)) + 1
    x0 = -(nx - 1) * dx / 2
    grid = Grid(nx, nx, dx, x0, x0, 0.9 * R)
    return StepSetup(grid, Ring(N, R), n_rays, ds, int(math.ceil(2.5 * R / ds)) + 2)


@functools.lru_cache(maxsize=None)
def water_tables(N=32, R=0.02, dx=0.4e-3, n_rays=180):
    from oracle.step import tables_for

    st = small_setup(N, R, dx, n_rays)
    c = np.full((st.grid.ny, st.grid.nx), C0)
    tb, ns = tables_for(c, st, 1)
    return st, tb
