"""Pins of the oracle's Eq. (7) combination, the prefactor of Eq. (8)-(10), and the
perfect-lattice behaviour of sigma as the broadening eta shrinks (Sec. II.B, Sec. II.C).

These fix what the other Kubo tests cannot: the conjugation and reality checks hold for any
sign pattern of the four energy pairs, and the synthetic currents give sigma no definite
sign, so neither a flipped cross term nor a wrong prefactor would show there.
"""

import numpy as np

import synthetic
from oracle import kkr, kubo


def _greenwood(H, j, e_fermi, eta, volume):
    """Greenwood's eigenstate form of the Kubo-Greenwood conductivity of independent electrons
    with Lorentzian-broadened delta functions (hbar = 1):
        sigma = (pi / V) sum_{m,n} |j_mn|^2 d(eF - e_m) d(eF - e_n),  d(x) = (eta / pi) / (x^2 + eta^2),
    with j_mn the current's matrix elements between eigenstates of H."""
    e, U = np.linalg.eigh(H)
    jm = U.conj().T @ j @ U
    d = (eta / np.pi) / ((e_fermi - e) ** 2 + eta ** 2)
    return (np.pi / volume) * np.einsum("mn,m,n->", np.abs(jm) ** 2, d, d)


def test_eq7_combination_and_prefactor_reproduce_greenwood():
    """Eq. (7)-(8) for a model with Hermitian H and current j: with G(z) = (z - H)^-1,
    sigma~(z1, z2) = -(1/(pi V)) Tr[j G(z1) j G(z2)] combined by the oracle's Eq. (7) must equal
    Greenwood's formula.  Since G(z-) = G(z+)^dagger, the four-term combination is
    (1/(pi V)) Tr[j Im G j Im G]; a flipped cross-term sign, a lost 1/4 or a wrong prefactor
    (sign or 1/pi) breaks the equality."""
    rng = np.random.default_rng(41)
    n = 8
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    H = 0.3 * (A + A.conj().T)
    B = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    j = B + B.conj().T
    e_fermi, volume = 0.2, 37.0
    for eta in (0.3, 0.05):
        G = {"+": np.linalg.inv((e_fermi + 1j * eta) * np.eye(n) - H),
             "-": np.linalg.inv((e_fermi - 1j * eta) * np.eye(n) - H)}
        tr = np.array([[np.trace(j @ G[z1] @ j @ G[z2]) for _ in range(3)] for (z1, z2) in kubo.COMBOS])
        got = kubo.combine(kubo.sigma_tilde(tr, volume))
        ref = _greenwood(H, j, e_fermi, eta, volume)
        assert ref > 0
        assert np.allclose(got, ref, rtol=1e-12, atol=0), (eta, got, ref)
    # every single-term change of the combination is caught
    for k in range(4):
        bad = np.array(kubo.SIGNS)
        bad[k] = -bad[k]
        alt = 0.25 * np.tensordot(bad, kubo.sigma_tilde(tr, volume), axes=1)
        assert not np.allclose(alt, ref, rtol=1e-3)


def test_lsms_sum_with_energy_independent_current_is_the_difference_form():
    """With one current for all four energy pairs, Eq. (7) applied to Eq. (10) factors as
    sigma = -(1/(pi V)) 1/4 sum_m sum_a Tr[J^m (tau^{ma}(+) - tau^{ma}(-)) J^a (tau^{am}(+) - tau^{am}(-))],
    the form Tr[j Im G j Im G] of the Kubo-Greenwood conductivity; the right side is formed here
    from the oracle's tau blocks directly, without the four pair sums."""
    w = synthetic.workload("bcc16")
    J1 = np.array(w["J"])
    for c in range(4):
        J1[:, c] = w["J"][:, 0]
    atoms = [0, 5, 11]
    eta = w["etas"][0]
    r = kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], J1, w["e_fermi"], eta, atoms=atoms)
    sp = np.asarray(w["species"])
    ptr, latom, _ = r["liz"]
    ref = np.zeros(3, dtype=complex)
    for i in atoms:
        tau = r["tau"][i]
        mem = latom[ptr[i]:ptr[i + 1]]
        drow = tau["row+"] - tau["row-"]
        dcol = tau["col+"] - tau["col-"]
        for mu in range(3):
            ref[mu] += np.trace(J1[sp[i], 0, mu][None] @ drow @ J1[sp[mem], 0, mu] @ dcol, axis1=1, axis2=2).sum()
    ref *= -0.25 / (np.pi * r["volume"])
    assert np.allclose(r["sigma"], ref, rtol=1e-12, atol=0)


def _pure_sigma(w, r_liz, eta, phase=None, J=None):
    """sigma of the pure crystal from one atom: by translation invariance every atom's Kubo sum
    equals atom 0's (pinned in the oracle's Kubo tests), so the outer sum of Eq. (10) is N
    times it."""
    ph = w["phase"] if phase is None else phase
    JJ = w["J"] if J is None else J
    o = kubo.sigma(w["pos"], w["cell"], r_liz, w["species"], ph, JJ, w["e_fermi"], eta, atoms=[0])
    st = kubo.sigma_tilde(o["per_atom"][0] * len(w["pos"]), o["volume"])
    return kubo.combine(st).real


def test_perfect_lattice_sigma_finite_as_eta_shrinks_with_differences_linear_in_eta():
    """Pure fcc crystal at a fixed LIZ (19 sites): the matrix 1 - t g of a finite cluster has no
    singularity on the real axis, so sigma(eta) stays finite as eta -> 0 and approaches its limit
    linearly: for eta = 5, 2, 1 mRy the successive differences stand in the ratio 3 : 1."""
    w = synthetic.workload("fcc32")
    s = [_pure_sigma(w, w["r_liz"], eta) for eta in (0.005, 0.002, 0.001)]
    assert np.all(np.isfinite(s))
    ratio = (s[0] - s[1]) / (s[1] - s[2])
    assert np.all((ratio > 2.7) & (ratio < 3.3)), ratio


def test_perfect_lattice_liz_convergence_length_grows_as_eta_shrinks():
    """Sec. II.C: in a perfect, weakly scattering crystal the pair terms of Eq. (10) decay as
    exp(-2 Im(kappa) r) with Im(kappa) ~ eta / (2 sqrt(eF)), so without broadening sigma keeps
    growing with the LIZ radius (it diverges linearly as eta -> 0) and with broadening it
    saturates over a length ~ 1/eta.  Pure fcc, phase shifts scaled by 0.3, one current for all
    energy pairs: the growth of sigma's pair part from r_LIZ = 1.1a (19 sites) to 1.5a (43 sites)
    must increase as eta is halved, from nearly saturated at 0.5 Ry."""
    w = synthetic.workload("fcc32")
    a = w["a"]
    ph = w["phase"] * 0.3
    J1 = np.array(w["J"])
    for c in range(4):
        J1[:, c] = w["J"][:, 0]
    growth = []
    for eta in (0.5, 0.25, 0.125):
        onsite = _pure_sigma(w, 0.5 * a, eta, ph, J1)  # LIZ = the atom alone: tau = t
        s1 = _pure_sigma(w, 1.1 * a, eta, ph, J1) - onsite
        s2 = _pure_sigma(w, 1.5 * a, eta, ph, J1) - onsite
        growth.append(s2[0] / s1[0] - 1.0)
    assert growth[0] < 0.1 and growth[0] < growth[1] < growth[2] and growth[2] > 0.2, growth


def test_single_site_cluster_in_closed_form():
    """An isolated atom (LIZ = itself): tau = t exactly, so Eq. (10) is a closed form in the
    t_l and the current; with a current coupling only s and p_x (mu = x), and
    J(z1, z2)_{s,px} = u_c, J(z1, z2)_{px,s} = v_c for pair c, the sum is
    s[c] = J(z2,z1)_{s,px} t1(z1) J(z1,z2)_{px,s} t0(z2) + J(z2,z1)_{px,s} t0(z1) J(z1,z2)_{s,px} t1(z2),
    sigma~ = -s / (pi V) and Eq. (7) combines the four pairs."""
    e_fermi, eta, vol = 0.65, 0.01, 123.0
    phase = np.array([[0.8, 0.2, 0.6, 0.01]])
    u = np.array([0.3 + 0.1j, -0.2 + 0.4j, 0.5 - 0.3j, 0.1 + 0.2j])
    v = np.array([-0.6 + 0.2j, 0.25 + 0.05j, -0.1 - 0.4j, 0.3 + 0.3j])
    J = np.zeros((1, 4, 3, 16, 16), dtype=complex)
    px = 3  # L = l^2 + l + m for (l, m) = (1, 1)
    J[0, :, 0, 0, px] = u
    J[0, :, 0, px, 0] = v
    r = kubo.sigma(np.zeros((1, 3)), None, 1.0, np.array([0]), phase, J, e_fermi, eta, volume=vol)
    _, _, kp, _ = kkr.energies(e_fermi, eta)
    t0p = -np.sin(0.8) * np.exp(0.8j) / kp
    t1p = -np.sin(0.2) * np.exp(0.2j) / kp
    t = {"+": (t0p, t1p), "-": (np.conj(t0p), np.conj(t1p))}
    idx = {"++": 0, "+-": 1, "-+": 2, "--": 3}
    sig = 0.0
    for z1, z2, sign in (("+", "+", 1), ("+", "-", -1), ("-", "+", -1), ("-", "-", 1)):
        c, crev = idx[z1 + z2], idx[z2 + z1]
        s = u[crev] * t[z1][1] * v[c] * t[z2][0] + v[crev] * t[z1][0] * u[c] * t[z2][1]
        sig += 0.25 * sign * (-s / (np.pi * vol))
    assert np.isclose(r["sigma"][0], sig, rtol=1e-13, atol=0)
    assert r["sigma"][1] == 0 and r["sigma"][2] == 0
