"""Pins of the oracle's special functions against libraries and closed forms."""

import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp
from sympy.physics.wigner import real_gaunt

from oracle import special


XS = np.array([0.05 + 0.0j, 0.3 + 0.001j, 4.53 + 0.003j, 9.7 + 0.02j, 13.1 + 0.0015j, 2.0 - 0.5j])


def test_hankel_vs_scipy_complex_argument():
    h = special.hankel1(6, XS)
    for l in range(7):
        ref = sp.spherical_jn(l, XS) + 1j * sp.spherical_yn(l, XS)
        assert np.allclose(h[l], ref, rtol=1e-12, atol=0)


def test_hankel_vs_mpmath_half_integer_order():
    for x in (0.7 + 0.004j, 5.3 + 0.01j, 12.0 + 0.002j):
        h = special.hankel1(6, np.array([x]))
        for l in range(7):
            ref = complex(mpmath.hankel1(l + 0.5, x) * mpmath.sqrt(mpmath.pi / (2 * x)))
            assert abs(h[l][0] - ref) <= 1e-13 * abs(ref)


def test_hankel_closed_forms_l0_l1():
    x = XS
    h = special.hankel1(1, x)
    assert np.allclose(h[0], np.exp(1j * x) / (1j * x), rtol=1e-14)
    assert np.allclose(h[1], -np.exp(1j * x) * (x + 1j) / x**2, rtol=1e-14)


def test_real_ylm_closed_forms():
    rng = np.random.default_rng(1)
    v = rng.normal(size=(50, 3))
    u = v / np.linalg.norm(v, axis=1, keepdims=True)
    x, y, z = u.T
    Y = special.real_ylm(2, v)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 0], 1 / math.sqrt(4 * math.pi))
    assert np.allclose(Y[:, 1], c1 * y)   # (1,-1)
    assert np.allclose(Y[:, 2], c1 * z)   # (1, 0)
    assert np.allclose(Y[:, 3], c1 * x)   # (1, 1)
    assert np.allclose(Y[:, 4], math.sqrt(15 / (4 * math.pi)) * x * y)
    assert np.allclose(Y[:, 5], math.sqrt(15 / (4 * math.pi)) * y * z)
    assert np.allclose(Y[:, 6], math.sqrt(5 / (16 * math.pi)) * (3 * z * z - 1))
    assert np.allclose(Y[:, 7], math.sqrt(15 / (4 * math.pi)) * x * z)
    assert np.allclose(Y[:, 8], math.sqrt(15 / (16 * math.pi)) * (x * x - y * y))


def test_real_ylm_vs_scipy_complex_harmonics():
    rng = np.random.default_rng(2)
    v = rng.normal(size=(40, 3))
    r = np.linalg.norm(v, axis=1)
    th = np.arccos(v[:, 2] / r)
    ph = np.arctan2(v[:, 1], v[:, 0])
    Y = special.real_ylm(6, v)
    for l in range(7):
        for m in range(-l, l + 1):
            yc = sp.sph_harm_y(l, abs(m), th, ph)  # Condon-Shortley phase included
            if m == 0:
                ref = yc.real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * yc.real
            else:
                ref = math.sqrt(2) * (-1) ** m * yc.imag
            assert np.allclose(Y[:, l * l + l + m], ref, atol=1e-13)


def test_real_ylm_orthonormal_on_fine_grid():
    # independent product grid far finer than the one inside gaunt_table
    xt, wt = np.polynomial.legendre.leggauss(40)
    ph = np.linspace(0, 2 * np.pi, 81)[:-1]
    st = np.sqrt(1 - xt**2)
    pts = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)), np.outer(xt, np.ones_like(ph))], -1)
    w = np.outer(wt, np.full(len(ph), 2 * np.pi / len(ph)))
    Y = special.real_ylm(6, pts.reshape(-1, 3))
    S = (Y * w.reshape(-1, 1)).T @ Y
    assert np.allclose(S, np.eye(49), atol=1e-13)


def test_gaunt_matches_sympy_real_gaunt():
    C = special.gaunt_table(3, 3, 6)
    n = 0
    for l1 in range(4):
        for m1 in range(-l1, l1 + 1):
            for l2 in range(4):
                for m2 in range(-l2, l2 + 1):
                    for l3 in range(7):
                        for m3 in range(-l3, l3 + 1):
                            ref = float(real_gaunt(l1, l2, l3, m1, m2, m3))
                            got = C[l1 * l1 + l1 + m1, l2 * l2 + l2 + m2, l3 * l3 + l3 + m3]
                            assert abs(got - ref) < 1e-13
                            n += ref != 0.0
    assert n == 708


def test_gaunt_product_rule_at_random_points():
    # Y_L Y_L' = sum_L'' C_{L L' L''} Y_L''  exactly (l'' <= l + l' <= 6)
    C = special.gaunt_table(3, 3, 6)
    rng = np.random.default_rng(3)
    v = rng.normal(size=(30, 3))
    Y3 = special.real_ylm(3, v)
    Y6 = special.real_ylm(6, v)
    lhs = Y3[:, :, None] * Y3[:, None, :]
    rhs = np.einsum("abc,pc->pab", C, Y6)
    assert np.allclose(lhs, rhs, atol=1e-13)


def test_gaunt_selection_rules():
    C = special.gaunt_table(3, 3, 6)
    for L1 in range(16):
        l1, m1 = special.lm_of(L1)
        for L2 in range(16):
            l2, m2 = special.lm_of(L2)
            for L3 in range(49):
                l3, m3 = special.lm_of(L3)
                if C[L1, L2, L3] != 0.0:
                    assert (l1 + l2 + l3) % 2 == 0
                    assert abs(l1 - l2) <= l3 <= l1 + l2
