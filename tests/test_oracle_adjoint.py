"""Pin of the oracle's d sigma / d phase against central finite differences of the oracle."""

import numpy as np

import synthetic
from oracle import adjoint, kubo


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(31)
    pos = np.array([[0, 0, 0], [4.1, 0.3, -0.2], [0.5, 4.4, 0.1], [-0.2, 0.6, 3.9], [3.7, 3.9, 0.4],
                    [7.9, 0.2, 0.3]])
    species = np.array([0, 1, 0, 1, 1, 0], dtype=np.int32)
    phase = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])[species] + rng.uniform(-0.05, 0.05, (6, 4))
    J = synthetic.current_matrices(2, rng)
    vol, r_liz, ef, eta = 400.0, 6.0, 0.65, 0.01
    dsig = np.array([0.7, -0.4, 1.3])
    g = adjoint.dsigma_dphase(pos, None, r_liz, species, phase, J, ef, eta, dsig, volume=vol)
    assert np.abs(g.imag).max() < 1e-12 * np.abs(g.real).max()

    def L(ph):
        return float(np.dot(dsig, kubo.sigma(pos, None, r_liz, species, ph, J, ef, eta, volume=vol)["sigma"].real))

    h = 1e-6
    fd = np.zeros((6, 4))
    for k in range(6):
        for l in range(4):
            p1 = phase.copy()
            p1[k, l] += h
            p2 = phase.copy()
            p2[k, l] -= h
            fd[k, l] = (L(p1) - L(p2)) / (2 * h)
    assert np.allclose(g.real, fd, rtol=0, atol=1e-7 * np.abs(fd).max())
    # the site outside everyone else's LIZ still contributes through its own LIZ
    assert np.abs(fd[5]).max() > 0


def test_restricted_gradient_equals_full_gradient_entries():
    """The (site, l) restriction used for the large gradient workload skips only LIZ that hold
    no listed site: the listed entries equal those of the unrestricted gradient."""
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    dsig = np.array([1.0, 0.0, 0.0])
    args = (w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta, dsig)
    full = adjoint.dsigma_dphase(*args)
    pairs = [(3, 0), (3, 2), (9, 1), (14, 3)]
    part = adjoint.dsigma_dphase(*args, pairs=pairs)
    for k, l in pairs:
        assert part[k, l] == full[k, l]
    mask = np.ones((16, 4), dtype=bool)
    for k, l in pairs:
        mask[k, l] = False
    assert not part[mask].any()
