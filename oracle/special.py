"""Angular and radial special functions for the free-electron propagator.

Part of the test oracle (test infrastructure only; see ``oracle/__init__``).

Conventions (the paper leaves them open; Sec. II.A only says L = (l, m)):

* Real spherical harmonics, channel index L = l*l + l + m, built from
  associated Legendre functions P_l^m WITHOUT the Condon-Shortley phase:
      m = 0 : Y_l0  = N_l0 P_l(cos t)
      m > 0 : Y_lm  = sqrt(2) N_lm P_l^m(cos t) cos(m p)
      m < 0 : Y_lm  = sqrt(2) N_l|m| P_l^|m|(cos t) sin(|m| p)
  with N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  So Y_{1,1} ~ +x,
  Y_{1,-1} ~ +y, Y_{1,0} ~ +z.
* Gaunt coefficients C[L, L', L''] = integral of Y_L Y_L' Y_L'' over the unit
  sphere, evaluated by a product quadrature (Gauss-Legendre in cos t, uniform
  trapezoid in p) that is exact for the polynomial degrees involved.
* Spherical Hankel functions of the first kind h_l = j_l + i y_l for complex
  argument, by upward recurrence from h_0(x) = -i e^{ix}/x and
  h_{-1}(x) = e^{ix}/x.
"""

import math

import numpy as np


def n_channels(lmax):
    return (lmax + 1) * (lmax + 1)


def lm_of(L):
    """Inverse of L = l*l + l + m."""
    l = int(math.isqrt(L))
    return l, L - l * l - l


def assoc_legendre_nocs(lmax, x):
    """P_l^m(x) for 0 <= m <= l <= lmax without the Condon-Shortley phase.

    Returns an array P[l, m, ...] (zero for m > l).  Standard recurrences:
    P_m^m = (2m-1)!! (1-x^2)^{m/2};  P_{m+1}^m = x (2m+1) P_m^m;
    (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m.
    """
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((lmax + 1, lmax + 1) + x.shape)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    for m in range(lmax + 1):
        dfact = 1.0
        for q in range(1, 2 * m, 2):
            dfact *= q
        P[m, m] = dfact * s**m
        if m + 1 <= lmax:
            P[m + 1, m] = x * (2 * m + 1) * P[m, m]
        for l in range(m + 2, lmax + 1):
            P[l, m] = ((2 * l - 1) * x * P[l - 1, m] - (l + m - 1) * P[l - 2, m]) / (l - m)
    return P


def real_ylm(lmax, vec):
    """Real spherical harmonics Y_L(r^) for direction vectors ``vec[..., 3]``.

    The vectors need not be normalised (only the direction is used).
    Returns array [..., (lmax+1)^2].
    """
    v = np.asarray(vec, dtype=np.float64)
    r = np.sqrt(np.sum(v * v, axis=-1))
    ct = v[..., 2] / r
    phi = np.arctan2(v[..., 1], v[..., 0])
    P = assoc_legendre_nocs(lmax, ct)
    out = np.zeros(v.shape[:-1] + (n_channels(lmax),))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            N = math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                y = N * P[l, 0]
            elif m > 0:
                y = math.sqrt(2.0) * N * P[l, am] * np.cos(am * phi)
            else:
                y = math.sqrt(2.0) * N * P[l, am] * np.sin(am * phi)
            out[..., l * l + l + m] = y
    return out


def sphere_quadrature(lmax_total):
    """Nodes/weights on the unit sphere exact for polynomials of degree lmax_total."""
    n_t = lmax_total // 2 + 2
    n_p = lmax_total + 2
    xt, wt = np.polynomial.legendre.leggauss(n_t)
    phis = 2.0 * math.pi * np.arange(n_p) / n_p
    st = np.sqrt(1.0 - xt * xt)
    X = np.outer(st, np.cos(phis))
    Y = np.outer(st, np.sin(phis))
    Z = np.outer(xt, np.ones(n_p))
    W = np.outer(wt, np.full(n_p, 2.0 * math.pi / n_p))
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1), W.ravel()


def gaunt_table(lmax1, lmax2, lmax3):
    """C[L1, L2, L3] = integral of Y_L1 Y_L2 Y_L3 over the sphere (real harmonics)."""
    nodes, w = sphere_quadrature(lmax1 + lmax2 + lmax3)
    Y1 = real_ylm(lmax1, nodes)
    Y2 = real_ylm(lmax2, nodes)
    Y3 = real_ylm(lmax3, nodes)
    wy12 = (w[:, None] * Y1)[:, :, None] * Y2[:, None, :]  # [q, L1, L2]
    C = np.tensordot(wy12, Y3, axes=([0], [0]))  # sum over quadrature nodes q
    C[np.abs(C) < 1e-14] = 0.0
    return C


def hankel1(lmax, x):
    """Spherical Hankel functions h_l(x) = j_l(x) + i y_l(x), l = 0..lmax, complex x.

    Upward recurrence h_{l+1} = (2l+1)/x h_l - h_{l-1} starting from
    h_0 = -i e^{ix}/x and h_{-1} = e^{ix}/x.  Returns array [lmax+1, ...].
    """
    x = np.asarray(x, dtype=np.complex128)
    out = np.zeros((lmax + 1,) + x.shape, dtype=np.complex128)
    e = np.exp(1j * x)
    hm1 = e / x
    h = -1j * e / x
    out[0] = h
    for l in range(lmax):
        hn = (2 * l + 1) / x * h - hm1
        hm1, h = h, hn
        out[l + 1] = h
    return out
