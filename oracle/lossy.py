"""Power-law absorption and dispersion of Szabo's model (oracle; test infrastructure only).

Section 2.2 of the paper:
  * Eq. szabo_dispersion_equation: the complex wavenumber k~ = omega/c + alpha [tan(pi y/2) + i]
    = k + i alpha with the power-law absorption alpha = alpha0 omega^y;
  * Eq. wave-number: its real part k = omega/c + alpha0 tan(pi y/2) omega^y = omega / c_p(omega);
  * Eq. complex-wavevector: k_i = (alpha / k) kvec is parallel to the ray, so the absorption
    along a ray (Eq. absorption) is the line integral of alpha;
Section 3.1, Eq. scattering-potential: Upsilon_m = omega c k~;
Section 3.4: d|kbar|/domega = 2 |cos(theta/2)| [1/c + y tan(pi y/2) omega^(y-1) alpha0];
Section 5, Eq. amplitude-abs-discretised: A_abs = exp(-int alpha ds) along the ray.

Units: alpha0 in Np (rad/s)^-y m^-1, so alpha = alpha0 omega^y is in Np/m.

Readings (where the paper leaves a choice):
  * the rays at omega are traced on the wavenumber map in units of k0 = omega/c0,
    n_omega = k/k0 = n_s + c0 tan(pi y/2) omega^(y-1) alpha0_s, with n_s = box_w(c0/c) and
    alpha0_s = box_w(alpha0): the box window of Section 6.3.2 applied to the wavenumber map,
    which is linear in both maps. The rays therefore depend on omega and are traced once per
    frequency; the travel time T = int n_omega ds / c0 gives the phase omega T = int k ds
    (Eq. phase-discretised);
  * A_abs = exp(-omega^y B) with B = int alpha0_s ds along the same ray, integrated by the
    trapezoid rule at the ray samples like the travel time and carried to the nodes and
    receivers by the same linear interpolation;
  * the geometric amplitude keeps Eq. attenuation_geom_reference (water's k0 at the
    reference point next to the transducer), and the speed ratio of Eq.
    amplitude-geom-discretised is the phase-speed ratio c_p(x)/c_p(x_1) = n_omega(x_1) /
    n_omega(x), which the transport equation with |grad phi| = k gives;
  * Upsilon_m and the back-projection weight use the model's c and the unsmoothed alpha0 at
    the node; the smoothing window only shapes the map the rays follow;
  * the expressions are arranged so that alpha0 = 0 gives the lossless values bit for bit:
    omega c k~ is written omega^2 [1 + omega^(y-1) c alpha0 (tan(pi y/2) + i)], a division
    by it as a division by omega^2 and then by the bracket, and 2 k dk/domega as
    2k/c + 2k y tan(pi y/2) omega^(y-1) alpha0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Absorption:
    """Power-law absorption of the medium: alpha0 map (ny, nx) and the exponent y."""

    alpha0: np.ndarray
    y: float


def tan_py(y: float) -> float:
    """tan(pi y / 2), the dispersion coefficient of Eqs. szabo_dispersion_equation and
    wave-number."""
    return math.tan(0.5 * math.pi * y)


def attenuation(omega, alpha0, y):
    """alpha = alpha0 omega^y (Np/m), the imaginary part of k~."""
    return alpha0 * omega ** y


def wavenumber(omega, c, alpha0, y):
    """Real part k = omega/c + alpha0 tan(pi y/2) omega^y (Eq. wave-number)."""
    return omega / c + alpha0 * tan_py(y) * omega ** y


def complex_wavenumber(omega, c, alpha0, y):
    """k~ = k + i alpha (Eq. szabo_dispersion_equation, second form)."""
    return wavenumber(omega, c, alpha0, y) + 1j * attenuation(omega, alpha0, y)


def tracing_index(n_s, alpha0_s, omega, y, c0):
    """Map the rays at omega follow, in units of k0: n_omega = n_s + c0 tan(pi y/2)
    omega^(y-1) alpha0_s (k = k0 n_omega with n_s = c0/c)."""
    return n_s + c0 * tan_py(y) * omega ** (y - 1.0) * alpha0_s


def relative_potential(omega, c, alpha0, y):
    """Upsilon_m / omega^2 = c k~ / omega = 1 + omega^(y-1) c alpha0 (tan(pi y/2) + i)."""
    return 1.0 + omega ** (y - 1.0) * c * alpha0 * (tan_py(y) + 1j)


def scattering_potential(omega, c, alpha0, y):
    """Upsilon_m = omega c k~ (Eq. scattering-potential), as omega^2 times
    relative_potential."""
    return omega ** 2 * relative_potential(omega, c, alpha0, y)


def dk_domega(omega, c, alpha0, y):
    """dk/domega = 1/c + y tan(pi y/2) omega^(y-1) alpha0, so that d|kbar|/domega =
    2 |cos(theta/2)| dk/domega (Section 3.4)."""
    return 1.0 / c + y * tan_py(y) * omega ** (y - 1.0) * alpha0


def absorption_factor(omega, B, y):
    """A_abs = exp(-omega^y B) with B = int alpha0 ds along the ray (Eq.
    amplitude-abs-discretised)."""
    return np.exp(-(omega ** y) * B)
