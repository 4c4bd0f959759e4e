"""Pins of the resistivity step and the LIZ-convergence fits (Sec. II.C, Eqs. (28)-(35)).

The oracle's fits are checked against the coefficients the paper prints (exact
recovery from curves drawn with them), against Eq. (29)'s closed form, and the
library's host-side fits against the oracle's on noisy data.
"""

import json
import os

import numpy as np
import pytest

from oracle import resistivity as O

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "liz_fit_coefficients.json")))["cases"]
R_ANG = np.linspace(12.0, 24.0, 7)  # angstrom, where the printed fits describe data


@pytest.mark.parametrize("case", CASES, ids=[c["case"] for c in CASES])
def test_fits_recover_printed_coefficients(case):
    rho_lo = case["c0"] / R_ANG + case["c1"]
    c0, c1 = O.fit_linear(R_ANG, rho_lo)
    assert abs(c0 - case["c0"]) <= 1e-10 * case["c0"] and abs(c1 - case["c1"]) <= 1e-10 * case["c0"]
    b1 = -case["b1_caption"]
    rho_up = O.model_upper(R_ANG, case["b0"], b1, 0.15)
    f0, f1 = O.fit_upper(R_ANG, rho_up, two_alpha=0.15)
    assert abs(f0 - case["b0"]) <= 1e-9 * case["b0"] and abs(f1 - b1) <= 1e-9 * abs(b1)


def test_caption_sign_reading():
    """Both printed bounds fit the same data, so over the fitted range they nearly coincide.
    With Eq. (33)'s plus sign and b1 = -(caption's number) they do (within 10 %); with the
    caption's number taken as b1 they differ by more than 20 % everywhere in that range."""
    r = np.linspace(16.0, 24.0, 200)
    for c in CASES:
        lo = c["c0"] / r + c["c1"]
        adopted = O.model_upper(r, c["b0"], -c["b1_caption"], 0.15)
        other = O.model_upper(r, c["b0"], c["b1_caption"], 0.15)
        assert np.abs(adopted / lo - 1).max() < 0.10, c["case"]
        assert np.abs(other / lo - 1).max() > 0.20, c["case"]
        assert c["c1"] <= c["b0"]  # Eq. (35) at 1/r_LIZ -> 0


def test_linear_fit_is_exact_on_eq29():
    """Eq. (29): sigma = 2 a1 alpha (r - r_c) / (1 + 2 alpha (r - r_c)) inverts to
    Eq. (31), rho = k / (2 alpha a1) + 1 / a1 with k = 1 / (r - r_c), exactly."""
    a1, alpha, rc = 3.5e-3, 0.01, 4.2
    r = np.linspace(10.0, 30.0, 9)
    x = 2 * alpha * (r - rc)
    sigma = a1 * x / (1 + x)
    slope, icpt = O.fit_linear(r, 1.0 / sigma, r_c=rc)
    assert np.isclose(slope, 1 / (2 * alpha * a1), rtol=1e-12) and np.isclose(icpt, 1 / a1, rtol=1e-12)


def test_resistivity_and_spin_sum():
    rng = np.random.default_rng(5)
    s = rng.standard_normal((3, 3)) * 0.1 + np.diag([2.0, 3.0, 4.0])
    rho = O.resistivity(s)
    assert np.allclose(rho @ s, np.eye(3), atol=1e-14)
    assert np.allclose(O.resistivity(np.diag([2.0, 4.0, 5.0])), np.diag([0.5, 0.25, 0.2]), rtol=1e-15)
    assert np.array_equal(O.spin_sum(s, s), 2 * s)
    assert np.isclose(O.TWO_ALPHA_UPPER_PER_BOHR * O.BOHR_PER_ANGSTROM, 0.15, rtol=1e-15)


def test_library_fits_match_oracle():
    """Host-side fits of the library (own closed forms and Gauss-Newton) against the oracle's
    library least-squares on noisy curves, and its 3 x 3 inverse against the oracle's."""
    from paper_2311_12134_amd import resistivity as R
    rng = np.random.default_rng(9)
    r = R_ANG * O.BOHR_PER_ANGSTROM
    for c in CASES:
        clean_lo = c["c0"] / R_ANG + c["c1"]
        noisy = clean_lo * (1 + 0.02 * rng.standard_normal(R_ANG.size))
        assert np.allclose(R.fit_linear(r, noisy), O.fit_linear(r, noisy), rtol=1e-10)
        clean_up = O.model_upper(R_ANG, c["b0"], -c["b1_caption"], 0.15)
        noisy = clean_up * (1 + 0.02 * rng.standard_normal(R_ANG.size))
        assert np.allclose(R.fit_upper(r, noisy), O.fit_upper(r, noisy), rtol=1e-8)
        assert np.allclose(R.fit_upper(r, clean_up), (c["b0"], -c["b1_caption"]), rtol=1e-9)
    s = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    assert np.allclose(R.invert3(s), O.resistivity(s), rtol=1e-13, atol=1e-15)
    with pytest.raises(ValueError):
        R.invert3(np.zeros((3, 3)))
    with pytest.raises(ValueError):
        R.fit_linear([5.0, 5.0], [1.0, 2.0])
