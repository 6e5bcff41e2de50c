"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the inversion's arithmetic: it draws sound-speed phantoms on a
Cartesian grid, unit complex Gaussian noise and random operands, all from fixed seeds, and
lists the workload configurations (ring, grid, frequencies, ray fan) as plain numbers.
Both the FP64 oracle and the HIP path receive what it returns as inputs.

The phantoms stand in for the digital breast phantom of the paper's experiments (Section 6.1:
water 1500 m/s, tissue 1470-1580 m/s, a ring of point transducers); nothing of that dataset
is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_WATER = 1500.0  # m/s, the medium outside the imaging region (Section 6.1)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One workload: ring of N point transducers (each emits and receives), square grid,
    frequency list, ray fan. Lengths in metres, frequencies in Hz."""

    name: str
    n_trans: int
    radius: float
    nx: int
    dx: float
    mask_radius: float
    freqs: tuple
    n_rays: int
    ds: float
    tau: float = 0.12
    phantom: str = "gaussian"
    phantom_seed: int = 1
    noise_seed: int = 2
    n_lesions: int = 3
    psi0: float = 0.0
    smooth_1mm: tuple = (1,)  # smoothing windows at 1 mm spacing, one per quartile of freqs

    @property
    def ny(self) -> int:
        return self.nx

    @property
    def x0(self) -> float:
        return -(self.nx - 1) * self.dx / 2.0

    @property
    def y0(self) -> float:
        return self.x0

    def max_steps(self) -> int:
        # chord of the ring plus a quarter for bent rays
        return int(math.ceil(2.5 * self.radius / self.ds)) + 2

    def smooth_window(self, freq_index: int) -> int:
        """Odd box-window width for the frequency with this index (windows given at 1 mm
        are scaled by 1 mm / dx and rounded down to the nearest odd integer)."""
        ws = self.smooth_1mm
        if len(ws) == 1 and ws[0] == 1:
            return 1
        q = min(len(ws) - 1, (freq_index * len(ws)) // max(1, len(self.freqs)))
        w = ws[q] * 1e-3 / self.dx
        return 2 * int(math.floor(w / 2.0)) + 1


# Ring of 64, 128^2 grid at 0.8 mm, one Gaussian inclusion, one frequency of 300 kHz.
SMALL = Workload(
    name="ring64_grid128",
    n_trans=64, radius=0.05, nx=128, dx=0.8e-3, mask_radius=0.045,
    freqs=(300e3,), n_rays=360, ds=0.2e-3, phantom="gaussian",
)

# Ring of 256, 512^2 grid at 0.45 mm, breast-like phantom, 16 frequencies 100-800 kHz.
MEDIUM = Workload(
    name="ring256_grid512",
    n_trans=256, radius=0.11, nx=512, dx=0.45e-3, mask_radius=0.099,
    freqs=tuple(np.linspace(100e3, 800e3, 16).tolist()), n_rays=720, ds=0.2e-3,
    phantom="breast", n_lesions=3, smooth_1mm=(13, 11, 9, 7),
)

# Clinical size: ring of 1024, 1024^2 grid at 0.22 mm, 32 frequencies 0.1-1.2 MHz.
LARGE = Workload(
    name="ring1024_grid1024",
    n_trans=1024, radius=0.11, nx=1024, dx=0.22e-3, mask_radius=0.099,
    freqs=tuple(np.linspace(100e3, 1.2e6, 32).tolist()), n_rays=1024, ds=0.2e-3,
    phantom="breast", n_lesions=10, smooth_1mm=(13, 11, 9, 7),
)

WORKLOADS = {w.name: w for w in (SMALL, MEDIUM, LARGE)}

# Serving mix: three scan classes on the 110 mm ring with one ray per transducer per
# transducer count (n_rays = N); 32 frequencies each from 100 kHz to the class's highest,
# about four grid spacings per wavelength in water at the top.
SERVE_CLASSES = tuple(
    Workload(name=f"serve_ring{n}_grid{nx}", n_trans=n, radius=0.11, nx=nx, dx=dx,
             mask_radius=0.099, freqs=tuple(np.linspace(100e3, fmax, 32).tolist()), n_rays=n,
             ds=0.2e-3, phantom="breast", n_lesions=lesions, smooth_1mm=(13, 11, 9, 7))
    for n, nx, dx, fmax, lesions in ((256, 256, 0.9e-3, 400e3, 3),
                                     (512, 512, 0.45e-3, 800e3, 3),
                                     (1024, 1024, 0.22e-3, 1.2e6, 10)))


@dataclasses.dataclass(frozen=True)
class ServeDraw:
    """One request of a serving run: scan class, phantom seed, number of steps, arrival (s)."""

    rid: int
    cls: int
    phantom_seed: int
    n_steps: int
    arrival: float


def serve_draws(n_requests: int = 64, seed: int = 5, rate: float | None = None,
                n_classes: int = 3, seeds_per_class: int = 3, min_steps: int = 8,
                max_steps: int = 32) -> list:
    """Seeded requests: class uniform, phantom seed from a pool of seeds_per_class per class,
    steps uniform in [min_steps, max_steps], Poisson arrivals at `rate` per second (unit
    exponential gaps scaled by 1 / rate, so one seed gives the same pattern at every rate;
    every request at time 0 if rate is None)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cls = rng.integers(0, n_classes, n_requests)
    pseed = 11 + rng.integers(0, seeds_per_class, n_requests)
    steps = rng.integers(min_steps, max_steps + 1, n_requests)
    gaps = rng.exponential(1.0, n_requests)
    t = np.cumsum(gaps) / rate if rate else np.zeros(n_requests)
    return [ServeDraw(i, int(cls[i]), int(pseed[i]), int(steps[i]), float(t[i]))
            for i in range(n_requests)]


def step_frequencies(n_steps: int, n_freqs: int) -> list:
    """Indices into a class's frequency list of a request with n_steps steps: spread evenly
    from the lowest to the highest, low to high."""
    if n_steps == 1:
        return [0]
    return [int(round(k * (n_freqs - 1) / (n_steps - 1))) for k in range(n_steps)]


def node_coords(nx: int, ny: int, dx: float, x0: float, y0: float):
    """Cartesian coordinates of the nodes, arrays of shape (ny, nx), x fastest."""
    xs = x0 + dx * np.arange(nx, dtype=np.float64)
    ys = y0 + dx * np.arange(ny, dtype=np.float64)
    return np.meshgrid(xs, ys, indexing="xy")


def water(nx: int, ny: int) -> np.ndarray:
    return np.full((ny, nx), C_WATER, dtype=np.float64)


def gaussian_inclusion(nx, ny, dx, x0, y0, seed=1, amp=45.0, sigma=8e-3,
                       centre_radius=20e-3, mask_radius=None) -> np.ndarray:
    """Water plus one Gaussian inclusion of +amp m/s, width sigma, centre drawn uniformly in a
    disk of radius centre_radius (PCG64 seed). Water outside mask_radius if given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = centre_radius * math.sqrt(rng.uniform())
    a = rng.uniform(0.0, 2.0 * math.pi)
    xc, yc = r * math.cos(a), r * math.sin(a)
    X, Y = node_coords(nx, ny, dx, x0, y0)
    c = C_WATER + amp * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2.0 * sigma ** 2))
    if mask_radius is not None:
        c[X ** 2 + Y ** 2 > mask_radius ** 2] = C_WATER
    return c


def _breast(nx, ny, dx, x0, y0, seed, n_lesions, mask_radius):
    """Sound speed (m/s) and absorption alpha0 (dB MHz^-y cm^-1) of the breast-like slice."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = node_coords(nx, ny, dx, x0, y0)
    a_ax = rng.uniform(60e-3, 80e-3)
    b_ax = rng.uniform(45e-3, 65e-3)
    rot = rng.uniform(0.0, math.pi)
    rc = 5e-3 * math.sqrt(rng.uniform())
    ac = rng.uniform(0.0, 2.0 * math.pi)
    cx, cy = rc * math.cos(ac), rc * math.sin(ac)
    cr, sr = math.cos(rot), math.sin(rot)

    def local(px, py):
        return ((px - cx) * cr + (py - cy) * sr, -(px - cx) * sr + (py - cy) * cr)

    U, V = local(X, Y)
    inside = (U / a_ax) ** 2 + (V / b_ax) ** 2 <= 1.0
    tissue = np.full_like(X, 1470.0)
    for _ in range(6):
        rr = 0.7 * math.sqrt(rng.uniform())
        th = rng.uniform(0.0, 2.0 * math.pi)
        bu, bv = rr * a_ax * math.cos(th), rr * b_ax * math.sin(th)
        sig = rng.uniform(5e-3, 12e-3)
        peak = rng.uniform(1520.0, 1560.0)
        tissue = np.maximum(tissue, 1470.0 + (peak - 1470.0)
                            * np.exp(-((U - bu) ** 2 + (V - bv) ** 2) / (2 * sig ** 2)))
    c = np.where(inside, tissue, C_WATER)
    c = gaussian_filter(c, sigma=2e-3 / dx, mode="nearest")
    # absorption: fat 0.45, rising to 0.8 with the glandular blobs; water 0
    a = np.where(inside, 0.45 + 0.35 * (tissue - 1470.0) / 90.0, 0.0)
    a = gaussian_filter(a, sigma=2e-3 / dx, mode="nearest")
    placed = []
    tries = 0
    while len(placed) < n_lesions and tries < 10000:
        tries += 1
        rad = rng.uniform(3e-3, 8e-3)
        rr = 0.75 * math.sqrt(rng.uniform())
        th = rng.uniform(0.0, 2.0 * math.pi)
        lu, lv = rr * a_ax * math.cos(th), rr * b_ax * math.sin(th)
        speed = rng.uniform(1560.0, 1580.0)
        if any(math.hypot(lu - pu, lv - pv) < rad + pr + 2e-3 for pu, pv, pr in placed):
            continue
        placed.append((lu, lv, rad))
        s = 0.5 * (1.0 - np.tanh((np.hypot(U - lu, V - lv) - rad) / 0.5e-3))
        c = c * (1.0 - s) + speed * s
        a = a * (1.0 - s) + 0.95 * s
    if mask_radius is not None:
        out = X ** 2 + Y ** 2 > mask_radius ** 2
        c[out] = C_WATER
        a[out] = 0.0
    return c, a


def breast_phantom(nx, ny, dx, x0, y0, seed=1, n_lesions=3, mask_radius=None) -> np.ndarray:
    """Breast-like slice: water 1500 m/s; a fat ellipse at 1470 m/s (semi-axes U[60,80] x
    U[45,65] mm, random rotation, centre within 5 mm); six glandular Gaussian blobs peaking
    at 1520-1560 m/s (sigma U[5,12] mm) inside 0.7 of the semi-axes; the map then smoothed by
    a Gaussian of sigma 2 mm; n_lesions disks of radius U[3,8] mm at 1560-1580 m/s with a
    0.5 mm tanh edge, not overlapping. Water outside mask_radius if given."""
    return _breast(nx, ny, dx, x0, y0, seed, n_lesions, mask_radius)[0]


def breast_absorption(nx, ny, dx, x0, y0, seed=1, n_lesions=3, mask_radius=None) -> np.ndarray:
    """Absorption coefficient alpha0 of the breast_phantom of the same arguments, in
    dB MHz^-y cm^-1 (the paper's range 0-1, Section 6.1): 0 in water, 0.45 in fat rising to
    0.8 with the glandular blobs (smoothed like the sound speed), 0.95 in the lesions."""
    return _breast(nx, ny, dx, x0, y0, seed, n_lesions, mask_radius)[1]


def gaussian_absorption(nx, ny, dx, x0, y0, seed=1, amp_db=1.0, sigma=8e-3,
                        centre_radius=20e-3, mask_radius=None) -> np.ndarray:
    """alpha0 (dB MHz^-y cm^-1) of amp_db exp(-r^2 / 2 sigma^2) centred on the inclusion that
    gaussian_inclusion draws from the same seed; 0 outside mask_radius if given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = centre_radius * math.sqrt(rng.uniform())
    a = rng.uniform(0.0, 2.0 * math.pi)
    xc, yc = r * math.cos(a), r * math.sin(a)
    X, Y = node_coords(nx, ny, dx, x0, y0)
    out = amp_db * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2.0 * sigma ** 2))
    if mask_radius is not None:
        out[X ** 2 + Y ** 2 > mask_radius ** 2] = 0.0
    return out


def db_to_neper(alpha_db, y: float):
    """Unit conversion of an absorption coefficient: dB MHz^-y cm^-1 to Np (rad/s)^-y m^-1
    (amplitude decibels: 1 dB = ln(10)/20 Np)."""
    return alpha_db * (math.log(10.0) / 20.0) * 100.0 * (2.0e6 * math.pi) ** (-y)


def linear_gradient(nx, ny, dx, x0, y0, c_a=C_WATER, gx=500.0, gy=0.0) -> np.ndarray:
    """c(x) = c_a + g . x on the whole grid (no water ring)."""
    X, Y = node_coords(nx, ny, dx, x0, y0)
    return c_a + gx * X + gy * Y


def phantom_for(w: Workload, seed: int | None = None) -> np.ndarray:
    seed = w.phantom_seed if seed is None else seed
    if w.phantom == "gaussian":
        return gaussian_inclusion(w.nx, w.ny, w.dx, w.x0, w.y0, seed=seed,
                                  mask_radius=w.mask_radius)
    if w.phantom == "breast":
        return breast_phantom(w.nx, w.ny, w.dx, w.x0, w.y0, seed=seed,
                              n_lesions=w.n_lesions, mask_radius=w.mask_radius)
    if w.phantom == "water":
        return water(w.nx, w.ny)
    raise ValueError(w.phantom)


def absorption_for(w: Workload, seed: int | None = None, y: float = 1.4) -> np.ndarray:
    """alpha0 map (Np (rad/s)^-y m^-1) matching phantom_for(w, seed): the absorption of the
    same breast-like slice, or a 1 dB MHz^-y cm^-1 peak on the Gaussian inclusion."""
    seed = w.phantom_seed if seed is None else seed
    if w.phantom == "gaussian":
        a = gaussian_absorption(w.nx, w.ny, w.dx, w.x0, w.y0, seed=seed,
                                mask_radius=w.mask_radius)
    elif w.phantom == "breast":
        a = breast_absorption(w.nx, w.ny, w.dx, w.x0, w.y0, seed=seed,
                              n_lesions=w.n_lesions, mask_radius=w.mask_radius)
    elif w.phantom == "water":
        a = np.zeros((w.ny, w.nx))
    else:
        raise ValueError(w.phantom)
    return db_to_neper(a, y)


def complex_noise(shape, seed) -> np.ndarray:
    """Circular complex Gaussian samples with E|z|^2 = 1 (PCG64 seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(tuple(shape) + (2,))
    return (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)


def real_uniform(shape, seed, lo=-1.0, hi=1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape)
