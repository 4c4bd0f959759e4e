"""Plain, slow FP64 CPU oracle for the LSMS tau-solve + Kubo-Greenwood hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg do.  It shares no code with the HIP library
(no kernels, headers, tables or helpers); both sides only see the same seeded
arrays produced by the ``synthetic`` input generators.

Everything is complex128 / float64 and written to be checked against the
paper by eye:

* ``special``  -- real spherical harmonics, Gaunt coefficients by quadrature,
                  spherical Hankel functions by recurrence (the ingredients of
                  the free-electron propagator g in Eq. (3)).
* ``liz``      -- local interaction zone of every atom (Sec. II.A, Fig. 1).
* ``kkr``      -- t-matrices, structure constants g, the matrix 1 - t g and the
                  tau blocks of Eq. (3)-(4).
* ``kubo``     -- the LSMS Kubo-Greenwood sum Eq. (10), the four-term
                  combination Eq. (7), and the all-site form Eq. (9).
* ``adjoint``  -- d sigma / d phase-shift by forward differentiation of Eq. (3)
                  through a dense inverse.
* ``resistivity`` -- rho = sigma^-1, the spin sum, and the LIZ-convergence fits
                  of Eqs. (31)-(34).

Every function is pinned by tests under ``tests/`` against closed forms,
library special functions, brute force and invariants of the equations.
"""

from . import special, liz, kkr, kubo, adjoint, resistivity  # noqa: F401
