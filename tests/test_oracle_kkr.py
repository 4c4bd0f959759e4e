"""Pins of the oracle's structure constants, t-matrices and tau blocks.

The structure constants are pinned by the free Green function itself (two-centre
expansion), tau by closed forms, the Dyson series of Eq. (5), brute force and the
symmetries the equations imply.
"""

import numpy as np
import pytest
import scipy.special as sp

from oracle import kkr, special

KP = np.sqrt(0.7 + 0.005j)
LSH = np.array([0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3])
PAR = np.diag((-1.0) ** LSH)


def _regular(lmax, kappa, x):
    ls = np.array([special.lm_of(L)[0] for L in range((lmax + 1) ** 2)])
    return sp.spherical_jn(ls, kappa * np.linalg.norm(x)) * special.real_ylm(lmax, x)


@pytest.mark.parametrize("pb", [np.array([3.1, -2.2, 4.0]), np.array([-5.4, 0.3, 0.1]), np.array([0.0, 0.0, 6.2])])
def test_g0_reproduces_free_green_function(pb):
    """-exp(ik|r-r'|)/(4 pi |r-r'|) = sum j_L(x) g^{ab}_{LL'} j_L'(x') for r = p_a + x, r' = p_b + x'."""
    lmax = 8
    pa = np.zeros(3)
    g = kkr.g0_block(pa - pb, KP, lmax)
    rng = np.random.default_rng(5)
    for _ in range(4):
        x = rng.normal(size=3)
        x *= 0.3 / np.linalg.norm(x)
        xp = rng.normal(size=3)
        xp *= 0.25 / np.linalg.norm(xp)
        d = np.linalg.norm(pa + x - pb - xp)
        exact = -np.exp(1j * KP * d) / (4 * np.pi * d)
        series = _regular(lmax, KP, x) @ g @ _regular(lmax, KP, xp)
        assert abs(series - exact) <= 1e-11 * abs(exact)


def test_g0_swave_block_closed_form():
    R = np.array([2.0, -3.0, 1.5])
    d = np.linalg.norm(R)
    g = kkr.g0_block(R, KP)
    assert abs(g[0, 0] - (-np.exp(1j * KP * d) / d)) < 1e-14


def test_g0_reciprocity_and_parity():
    R = np.array([3.3, 1.1, -2.7])
    g = kkr.g0_block(R, KP)
    gm = kkr.g0_block(-R, KP)
    assert np.allclose(g, gm.T, rtol=0, atol=1e-14 * np.abs(g).max())          # g_LL'(R) = g_L'L(-R)
    assert np.allclose(gm, PAR @ g @ PAR, rtol=0, atol=1e-14 * np.abs(g).max())  # g(-R) = (-1)^{l+l'} g(R)


def test_g0_at_z_minus_is_parity_conjugate():
    _, _, kp, km = kkr.energies(0.7, 0.005)
    R = np.array([-1.2, 4.4, 2.0])
    gp = kkr.g0_block(R, kp)
    gmn = kkr.g0_block(R, km)
    assert np.allclose(gmn, PAR @ np.conj(gp) @ PAR, rtol=0, atol=1e-14 * np.abs(gp).max())


def test_energies_sheet():
    zp, zm, kp, km = kkr.energies(0.65, 0.002)
    assert kp.imag > 0 and abs(kp * kp - zp) < 1e-15
    assert abs(km * km - zm) < 1e-15 and km == -np.conj(kp)


def test_t_matrix_outside_solution():
    """j_l - i kappa t_l h_l = e^{i delta} (cos delta j_l - sin delta y_l)."""
    delta = np.array([0.9, 0.3, 0.05, 0.005])
    tp, tm = kkr.t_matrix(delta, KP)
    for r in (0.7, 3.0, 8.0):
        x = KP * r
        for l in range(4):
            j = sp.spherical_jn(l, x)
            y = sp.spherical_yn(l, x)
            lhs = j - 1j * KP * tp[l] * (j + 1j * y)
            rhs = np.exp(1j * delta[l]) * (np.cos(delta[l]) * j - np.sin(delta[l]) * y)
            assert abs(lhs - rhs) < 1e-14
    assert np.allclose(tm, np.conj(tp))


def _cluster(n, seed, spacing=5.0):
    rng = np.random.default_rng(seed)
    p = [np.zeros(3)]
    while len(p) < n:
        c = rng.uniform(-spacing, spacing, size=3)
        if min(np.linalg.norm(c - q) for q in p) > 2.5:
            p.append(c)
    return np.array(p)


def test_single_site_tau_is_t():
    t = kkr.t_matrix(np.array([0.8, 0.2, 0.6, 0.01]), KP)[0]
    M = kkr.kkr_matrix(np.zeros((1, 3)), t[None, :], KP)
    col, row = kkr.tau_blocks(M, t[None, :])
    assert np.allclose(col[0], np.diag(kkr.expand_t(t)), atol=1e-15)
    assert np.allclose(row[0], np.diag(kkr.expand_t(t)), atol=1e-15)


def test_two_site_swave_closed_form():
    R = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, -4.0]])
    delta = np.array([[0.7, 0, 0, 0], [0.4, 0, 0, 0]])
    t = kkr.t_matrix(delta, KP)[0]
    M = kkr.kkr_matrix(R, t, KP)
    col, row = kkr.tau_blocks(M, t)
    d = np.linalg.norm(R[1])
    g = -np.exp(1j * KP * d) / d
    a, b = 1 / t[0, 0], 1 / t[1, 0]
    det = a * b - g * g
    assert abs(col[0][0, 0] - b / det) < 1e-13 * abs(b / det)
    assert abs(col[1][0, 0] - g / det) < 1e-13 * abs(g / det)
    assert abs(row[1][0, 0] - g / det) < 1e-13 * abs(g / det)
    assert np.abs(col[:, 1:, :]).max() == 0 and np.abs(col[:, :, 1:]).max() == 0


def test_dyson_series_weak_scattering():
    """Eq. (5): tau = t + t g t + t g t g t + O(t^4) when every phase shift is scaled by lam."""
    P = _cluster(4, 11)
    base = np.array([[0.8, 0.2, 0.6, 0.01]] * 4) * np.linspace(0.8, 1.2, 4)[:, None]
    errs = []
    for lam in (1e-2, 5e-3):
        t = kkr.t_matrix(base * lam, KP)[0]
        M = kkr.kkr_matrix(P, t, KP)
        col, _ = kkr.tau_blocks(M, t)
        G = kkr.g0_matrix(P, KP)
        T = np.diag(kkr.expand_t(t).reshape(-1))
        series = T + T @ G @ T + T @ G @ T @ G @ T
        err = np.abs(col.reshape(-1, 16) - series[:, :16]).max() / np.abs(T).max()
        errs.append(err)
    # third-order remainder relative to t: O(lam^3) -> ratio ~ 8 when lam halves
    assert errs[0] < 1e-4 and errs[0] / errs[1] > 6.0


def test_tau_matches_brute_force_inverse():
    P = _cluster(6, 3)
    delta = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]] * 3)
    for kappa in kkr.energies(0.65, 0.002)[2:]:
        t = kkr.t_matrix(delta, KP)[0]
        M = kkr.kkr_matrix(P, t, kappa)
        col, row = kkr.tau_blocks(M, t)
        Tinv = np.diag(1.0 / kkr.expand_t(t).reshape(-1))
        tau = np.linalg.inv(Tinv - kkr.g0_matrix(P, kappa))
        nm = len(P)
        full = tau.reshape(nm, 16, nm, 16)
        assert np.allclose(col, full[:, :, 0, :], atol=1e-12 * np.abs(tau).max())
        assert np.allclose(row, full[0].transpose(1, 0, 2), atol=1e-12 * np.abs(tau).max())


def test_tau_reciprocity_and_energy_conjugation():
    P = _cluster(7, 4)
    delta = np.array([[0.9, 0.3, 0.05, 0.005]] * 7)
    _, _, kp, km = kkr.energies(0.7, 0.005)
    tp, tm = kkr.t_matrix(delta, kp)
    out = kkr.atom_tau(P, tp, tm, kp, km)
    for e in "+-":
        assert np.allclose(out["row" + e], out["col" + e].transpose(0, 2, 1), atol=1e-13)
    assert np.allclose(out["col-"], PAR @ np.conj(out["col+"]) @ PAR, atol=1e-13)


def test_tau_invariant_under_member_permutation():
    P = _cluster(6, 8)
    delta = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]] * 3)
    t = kkr.t_matrix(delta, KP)[0]
    col, _ = kkr.tau_blocks(kkr.kkr_matrix(P, t, KP), t)
    perm = np.array([0, 4, 2, 5, 1, 3])
    col2, _ = kkr.tau_blocks(kkr.kkr_matrix(P[perm], t[perm], KP), t[perm])
    assert np.allclose(col2, col[perm], atol=1e-13)
