"""Pins of the closed-form helpers against the paper's Sec. 3.

The helpers in oracle/analytic.py feed the torus tests, so they are pinned
here independently: determinants of the printed amplification matrices
against the printed characteristic polynomials, the printed small-c expansion
against numerically found roots, and the constants printed in the paper
(tests/golden/paper_constants.txt).
"""
import os

import numpy as np
import pytest

from oracle import analytic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            out[k.strip()] = float(v)
    return out


def _det_poly(Mx, lam):
    return np.linalg.det(Mx - lam * np.eye(Mx.shape[0]))


@pytest.mark.parametrize("c,theta", [(0.3, 0.14), (1.1, 0.14), (0.7, 0.0), (1.5, 0.3)])
def test_se_polynomial_is_det_of_eq3_7(c, theta):
    for lam in (0.3 + 0.2j, -0.7 + 1.1j, 1.3):
        p = np.polyval(analytic.se_char_poly_coeffs(c, theta)[::-1], lam)
        assert abs(p - _det_poly(analytic.se_matrix(c, theta), lam)) < 1e-12


@pytest.mark.parametrize("c,theta,alpha", [(0.4, 0.6, 0.7), (2.0, 1.0, 1.0), (5.0, 0.55, 0.8)])
def test_si_polynomial_is_det_of_eq3_3(c, theta, alpha):
    for lam in (0.3 + 0.2j, -0.7 + 1.1j):
        p = np.polyval(analytic.si_char_poly_coeffs(c, theta, alpha)[::-1], lam)
        assert abs(p - _det_poly(analytic.si_matrix(c, theta, alpha), lam)) < 1e-12


def test_sesm_polynomial_is_det_of_eq3_5():
    b, z = 0.281105, 0.01
    g = 0.05
    d = 0.7
    for c in (0.2, 0.9):
        for lam in (0.3 + 0.2j, -0.7 + 1.1j, 0.9 - 0.1j):
            p = np.polyval(analytic.sesm_char_poly_coeffs(c, b, d, g, z)[::-1], lam)
            assert abs(p - _det_poly(analytic.sesm_matrix(c, b, d, g, z), lam)) < 1e-12


@pytest.mark.parametrize("theta", [0.0, 0.14, 0.3])
def test_se_small_c_expansion_eqdp_5(theta):
    m, n, q = analytic.se_expansion(theta)
    errs = []
    for c in (0.08, 0.04, 0.02):
        lam = analytic.se_physical_root(c, theta)
        errs.append(abs(lam - (1 + m * c + n * c * c + q * c ** 3)))
    # remainder is at least fourth order: halving c divides it by >= ~16
    assert errs[0] < 1e-4
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12


@pytest.mark.parametrize("theta", [0.0, 0.14, 0.3])
def test_se_dissipation_eqdp_4(theta):
    chi = analytic.se_chi(theta)
    for c in (1e-2, 5e-3):
        lam = analytic.se_physical_root(c, theta)
        assert abs(abs(lam) - (1 - chi * c * c)) < 5 * c ** 4
    # exact: |lambda|^2 = det = 1 - theta c^2 for the complex pair
    for c in (0.2, 1.0, 1.45):   # complex pair while c < 2/(1+theta)
        lam = analytic.se_physical_root(c, theta)
        assert abs(abs(lam) ** 2 - (1 - theta * c * c)) < 1e-13


@pytest.mark.parametrize("theta", [0.05, 0.14, 0.3])
def test_se_stability_limit(theta):
    cl = analytic.se_stability_limit(theta)
    assert np.max(np.abs(analytic.se_eigs(cl * (1 - 1e-6), theta))) <= 1.0
    assert np.max(np.abs(analytic.se_eigs(cl * (1 + 1e-6), theta))) > 1.0


def test_paper_constants_consistent():
    """theta = 0.14 for SE gives the chi = 0.07 used for all schemes in Fig. 2."""
    k = _golden()
    assert abs(analytic.se_chi(k["theta_se"]) - k["chi_fig2"]) < 1e-15
    # barotropic substep lengths quoted for the channel and global runs
    assert abs(k["tau_channel"] / k["M_channel"] - k["dts_channel"]) < 1e-12
    assert abs(k["tau_global"] / k["M_global"] - k["dts_global"]) < 1e-12
    # channel: c_p = 200 m/s crosses a 10 km cell in less than 50 s
    assert k["dx_channel"] / k["cp_channel"] <= 50.0


def test_sesm_parameters_give_printed_dissipation():
    """eqdp_6 (without O(c^3) phase accuracy) with chi = 0.07: numerical chi ~ 0.07."""
    k = _golden()
    chi, beta = k["chi_fig2"], k["beta_sesm"]
    zeta = 0.010 - 0.135 * chi
    gamma = 0.083 - 0.514 * chi
    delta = 2 * chi + gamma + 2 * zeta + 0.5      # eq. (eqdp_4), SESM line
    c = 1e-2
    roots = np.roots(analytic.sesm_char_poly_coeffs(c, beta, delta, gamma, zeta)[::-1])
    lam = roots[np.argmin(np.abs(roots - np.exp(1j * c)))]
    chi_num = (1 - abs(lam)) / c ** 2
    assert abs(chi_num - chi) < 1e-3


def test_fig2_amplitude_per_baroclinic_step():
    """Fig. 2 setting (M = 30, chi = 0.07): amplitude after M substeps is (1 - theta (c/M)^2)^(M/2)."""
    for c in (0.5, 2.0, 10.0, 30.0):
        amp, ph = analytic.per_step_response(c, 30, 0.14)
        assert abs(amp - (1 - 0.14 * (c / 30) ** 2) ** 15) < 1e-13
    # phase error is third order in the substep Courant number: M (c/M)^3 scale
    _, ph1 = analytic.per_step_response(0.5, 30, 0.14)
    _, ph2 = analytic.per_step_response(0.25, 30, 0.14)
    assert 7.0 < ph1 / ph2 < 9.0
