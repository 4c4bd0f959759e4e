"""Pins of the oracle's LIZ construction and Kubo-Greenwood sums."""

import numpy as np
import pytest

import synthetic
from oracle import kkr, kubo, liz


@pytest.mark.parametrize("lat,ncell,rfac,count", [
    ("fcc", 2, 1.1, 19), ("fcc", 4, 1.95, 135), ("bcc", 3, 1.5, 27), ("bcc", 5, 2.2, 89), ("bcc", 3, 1.6, 27)])
def test_liz_shell_counts(lat, ncell, rfac, count):
    a = 6.0
    pos, cell = (synthetic.fcc_supercell if lat == "fcc" else synthetic.bcc_supercell)(a, ncell)
    ptr, atoms, disp = liz.build_liz(pos, cell, rfac * a)
    sizes = np.diff(ptr)
    assert (sizes == count).all()


def test_liz_order_and_images():
    w = synthetic.workload("fcc32")
    ptr, atoms, disp = liz.build_liz(w["pos"], w["cell"], w["r_liz"])
    for i in range(len(w["pos"])):
        d = disp[ptr[i]:ptr[i + 1]]
        a = atoms[ptr[i]:ptr[i + 1]]
        assert a[0] == i and np.all(d[0] == 0)
        r = np.linalg.norm(d, axis=1)
        assert np.all(np.diff(r) >= -1e-9)
        # the displacement really is an image of that atom
        img = w["pos"][i] + d - w["pos"][a]
        frac = img / w["cell"][0, 0]
        assert np.allclose(frac, np.round(frac), atol=1e-12)
    # a 2x2x2 fcc box is smaller than the LIZ diameter: images of one atom recur
    a0 = atoms[ptr[0]:ptr[1]]
    assert len(set(a0.tolist())) < len(a0)


def test_liz_open_cluster_and_coincident_sites():
    pos = np.array([[0, 0, 0], [3.0, 0, 0], [0, 4.0, 0], [10.0, 0, 0]])
    ptr, atoms, disp = liz.build_liz(pos, None, 5.5)
    assert list(np.diff(ptr)) == [3, 3, 3, 1]
    with pytest.raises(ValueError):
        liz.build_liz(np.array([[0, 0, 0], [0, 0, 0.0]]), None, 2.0)


@pytest.fixture(scope="module")
def fcc32_result():
    w = synthetic.workload("fcc32")
    r = kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], w["etas"][0])
    return w, r


def test_sigma_tilde_conjugation_and_real_sigma(fcc32_result):
    w, r = fcc32_result
    st = r["sigma_tilde"]
    assert np.allclose(st[3], np.conj(st[0]), rtol=1e-12, atol=0)
    assert np.allclose(st[2], np.conj(st[1]), rtol=1e-12, atol=0)
    s = r["sigma"]
    assert np.all(np.abs(s.imag) <= 1e-12 * np.abs(s.real))


def test_cubic_isotropy_pure_fcc(fcc32_result):
    w, r = fcc32_result
    s = r["sigma"].real
    assert np.allclose(s, s[0], rtol=1e-11)


def test_translation_invariance_pure_crystal(fcc32_result):
    w, r = fcc32_result
    per = np.array([r["per_atom"][i] for i in range(32)])
    assert np.allclose(per, per[0], rtol=1e-10, atol=1e-12 * np.abs(per[0]).max())


def test_rotation_covariance_alloy():
    w = synthetic.workload("bcc16")
    args = (w["species"], w["phase"], w["J"], w["e_fermi"], w["etas"][0])
    r0 = kubo.sigma(w["pos"], w["cell"], w["r_liz"], *args)
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])  # +90 deg about z
    r1 = kubo.sigma(w["pos"] @ Rz.T, w["cell"] @ Rz.T, w["r_liz"], *args)
    s0, s1 = r0["sigma"].real, r1["sigma"].real
    assert abs(s0[0] - s0[1]) > 1e-6 * abs(s0[0])  # anisotropic sample, so the check bites
    assert np.allclose(s1, s0[[1, 0, 2]], rtol=1e-10)


def test_lsms_sum_equals_all_site_form_on_closed_cluster():
    """Eq. (10) with a LIZ covering the whole cluster equals Eq. (9) with one global inverse."""
    rng = np.random.default_rng(21)
    pos = np.array([[0, 0, 0], [4.1, 0.3, -0.2], [0.5, 4.4, 0.1], [-0.2, 0.6, 3.9], [3.7, 3.9, 0.4]])
    species = np.array([0, 1, 0, 1, 1], dtype=np.int32)
    phase = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])[species]
    J = synthetic.current_matrices(2, rng)
    vol = 500.0
    r10 = kubo.sigma(pos, None, 50.0, species, phase, J, 0.65, 0.01, volume=vol)
    r9 = kubo.sigma_all_sites(pos, species, phase, J, 0.65, 0.01, vol)
    assert np.allclose(r10["sigma_tilde"], r9["sigma_tilde"], rtol=1e-11)


def test_born_limit():
    """All phase shifts scaled by lam -> 0: only the a = 0 term survives, error O(lam^2)."""
    w = synthetic.workload("bcc16")
    atoms = [0, 5]
    errs = []
    for lam in (1e-2, 5e-3):
        ph = w["phase"] * lam
        r = kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], ph, w["J"], w["e_fermi"], w["etas"][0],
                       atoms=atoms)
        _, _, kp, km = kkr.energies(w["e_fermi"], w["etas"][0])
        tp, tm = kkr.t_matrix(ph, kp)
        tt = {"+": tp, "-": tm}
        born = np.zeros((4, 3), dtype=complex)
        for i in atoms:
            sp = w["species"][i]
            for c, (z1, z2) in enumerate(kubo.COMBOS):
                crev = kubo.COMBO_INDEX[(z2, z1)]
                for mu in range(3):
                    born[c, mu] += np.trace(w["J"][sp, crev, mu] @ np.diag(kkr.expand_t(tt[z1][i]))
                                            @ w["J"][sp, c, mu] @ np.diag(kkr.expand_t(tt[z2][i])))
        tot = sum(r["per_atom"][i] for i in atoms)
        errs.append(np.abs(tot - born).max() / np.abs(born).max())
    assert errs[0] < 1e-1 and 3.0 < errs[0] / errs[1] < 5.0


def test_sigma_converges_as_eta_shrinks():
    """At fixed LIZ, sigma(eta) tends to a finite limit; differences shrink with eta."""
    w = synthetic.workload("bcc16")
    vals = []
    for eta in (0.008, 0.004, 0.002):
        r = kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                       atoms=[0, 1, 2, 3])
        vals.append(r["sigma"].real)
    d1 = np.abs(vals[0] - vals[1]).max()
    d2 = np.abs(vals[1] - vals[2]).max()
    assert d2 < d1 and np.all(np.isfinite(vals))


def test_tensor_diagonal_equals_diagonal_sums():
    w = synthetic.workload("bcc16")
    args = (w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], w["etas"][0])
    rd = kubo.sigma(*args, atoms=[0, 3])
    rt = kubo.sigma(*args, atoms=[0, 3], tensor=True)
    assert rt["sigma_tilde"].shape == (4, 3, 3) and rt["sigma"].shape == (3, 3)
    diag = np.stack([rt["sigma_tilde"][:, m, m] for m in range(3)], axis=1)
    assert np.allclose(diag, rd["sigma_tilde"], rtol=1e-13, atol=0)
    off = rt["sigma_tilde"][:, 0, 1]
    assert np.abs(off).max() > 1e-3 * np.abs(diag).max()  # random currents: off-diagonal terms are not small


def test_tensor_lsms_sum_equals_all_site_form_on_closed_cluster():
    """Eq. (10) and Eq. (9) agree for every (mu, nu) when the LIZ spans the cluster."""
    rng = np.random.default_rng(22)
    pos = np.array([[0, 0, 0], [4.1, 0.3, -0.2], [0.5, 4.4, 0.1], [-0.2, 0.6, 3.9]])
    species = np.array([0, 1, 1, 0], dtype=np.int32)
    phase = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])[species]
    J = synthetic.current_matrices(2, rng)
    r10 = kubo.sigma(pos, None, 50.0, species, phase, J, 0.65, 0.01, volume=400.0, tensor=True)
    r9 = kubo.sigma_all_sites(pos, species, phase, J, 0.65, 0.01, 400.0, tensor=True)
    assert np.allclose(r10["sigma_tilde"], r9["sigma_tilde"], rtol=1e-11)
    # Eq. (9) alone: cyclic trace + relabelling m <-> n give sigma~_{mu nu}(z1, z2) = sigma~_{nu mu}(z2, z1)
    st = r9["sigma_tilde"]
    for c, (z1, z2) in enumerate(kubo.COMBOS):
        assert np.allclose(st[c], st[kubo.COMBO_INDEX[(z2, z1)]].T, rtol=1e-11)


def test_tensor_places_mu_on_the_centre_current():
    """Eq. (10) puts mu on J^{m mu} (centre atom) and nu on J^{n nu} (LIZ member).

    Species A loses its y current and species B its x current; with the outer sum
    over A atoms only, s_yx vanishes exactly, and s_xy (the B members' terms) is what
    the diagonal sum gains when B's x slot is given B's y current.
    """
    w = synthetic.workload("bcc16")
    sp = np.asarray(w["species"])
    A = int(sp[0])
    B = 1 - A
    centres = [int(i) for i in np.nonzero(sp == A)[0][:2]]
    J1 = np.array(w["J"])
    J1[A, :, 1] = 0.0
    J1[B, :, 0] = 0.0
    J2 = J1.copy()
    J2[B, :, 0] = w["J"][B, :, 1]
    base = (w["pos"], w["cell"], w["r_liz"], sp, w["phase"])
    s1 = kubo.sigma(*base, J1, w["e_fermi"], w["etas"][0], atoms=centres, tensor=True)["sigma_tilde"]
    s2 = kubo.sigma(*base, J2, w["e_fermi"], w["etas"][0], atoms=centres)["sigma_tilde"]
    assert np.all(s1[:, 1, 0] == 0)
    assert np.abs(s1[:, 0, 1]).max() > 1e-3 * np.abs(s1[:, 0, 0]).max()
    assert np.allclose(s2[:, 0], s1[:, 0, 0] + s1[:, 0, 1], rtol=1e-12)
