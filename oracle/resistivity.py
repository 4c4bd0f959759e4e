"""Resistivity from the conductivity tensor and the LIZ-convergence fits.

Part of the test oracle (test infrastructure only; see ``oracle/__init__``).

* Sec. II.C: the conductivity tensor of Eqs. (7) and (10) is inverted to give the
  resistivity, rho = sigma^-1 (a 3 x 3 matrix inverse).
* Spin: in a collinear spin-polarized calculation the two spin channels are
  computed separately (each with its own t-matrices) and their conductivities
  added before the inversion (Sec. IV, Fe-Si).
* Eq. (31) / Eq. (34): rho = c0 / (r_LIZ - r_c) + c1, linear in k = 1/(r_LIZ - r_c);
  the lower bound takes r_c = 0, and c1 is the value extrapolated to 1/r_LIZ -> 0.
* Eq. (32) / Eq. (33): rho = b0 / (1 + b1 exp(-2 alpha r_LIZ)) at a fixed 2 alpha
  (0.15 per angstrom for the upper bound); b0 is the extrapolated value.

Readings (the paper prints coefficients but not how it fitted them): both fits
are ordinary least squares in rho itself, the quantity the figures plot; the
linear one through ``numpy.linalg.lstsq``, the exponential one through
``scipy.optimize.least_squares`` started from the exact solution of Eq. (24)'s
form sigma = a1 + a0 exp(-2 alpha r) on the first and last points.  The figure
captions write the upper bound as b0 / (1 - b1 e^{-0.15 r}); Eq. (33) has a plus
sign, which is kept, so a caption's b1 appears here with the opposite sign.
Lengths in the caller's unit; ``TWO_ALPHA_UPPER_PER_BOHR`` converts 0.15 / angstrom.
"""

import numpy as np
from scipy import optimize

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
TWO_ALPHA_UPPER_PER_ANGSTROM = 0.15
TWO_ALPHA_UPPER_PER_BOHR = TWO_ALPHA_UPPER_PER_ANGSTROM / BOHR_PER_ANGSTROM


def resistivity(sigma):
    """rho = sigma^-1 of a real 3 x 3 conductivity tensor (Sec. II.C)."""
    return np.linalg.inv(np.asarray(sigma, dtype=np.float64))


def spin_sum(sigma_up, sigma_down):
    """Collinear spin: the two channels' conductivities add (Sec. IV)."""
    return np.asarray(sigma_up, dtype=np.float64) + np.asarray(sigma_down, dtype=np.float64)


def fit_linear(r_liz, rho, r_c=0.0):
    """Eq. (31) / (34): least-squares (c0, c1) of rho = c0 / (r_LIZ - r_c) + c1."""
    k = 1.0 / (np.asarray(r_liz, dtype=np.float64) - r_c)
    A = np.stack([k, np.ones_like(k)], axis=1)
    (c0, c1), *_ = np.linalg.lstsq(A, np.asarray(rho, dtype=np.float64), rcond=None)
    return float(c0), float(c1)


def model_upper(r_liz, b0, b1, two_alpha):
    """Eq. (32): b0 / (1 + b1 exp(-2 alpha r_LIZ))."""
    return b0 / (1.0 + b1 * np.exp(-two_alpha * np.asarray(r_liz, dtype=np.float64)))


def fit_upper(r_liz, rho, two_alpha=TWO_ALPHA_UPPER_PER_BOHR):
    """Eq. (32) / (33) at fixed 2 alpha: least-squares (b0, b1) in rho."""
    r = np.asarray(r_liz, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    # start: sigma = a1 + a0 e^{-2 alpha r} through the first and last points (Eq. (24)'s form)
    e0, e1 = np.exp(-two_alpha * r[0]), np.exp(-two_alpha * r[-1])
    s0, s1 = 1.0 / rho[0], 1.0 / rho[-1]
    a0 = (s0 - s1) / (e0 - e1)
    a1 = s0 - a0 * e0
    x0 = np.array([1.0 / a1, a0 / a1])
    res = optimize.least_squares(lambda x: model_upper(r, x[0], x[1], two_alpha) - rho, x0,
                                 xtol=1e-15, ftol=1e-15, gtol=1e-15)
    return float(res.x[0]), float(res.x[1])
