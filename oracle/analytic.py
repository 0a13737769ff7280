"""Closed forms from Sec. 3 of the paper (1D prototype, eq. (eq3_1)).

TEST INFRASTRUCTURE ONLY.  Amplification matrices eq. (eq3_3), (eq3_5),
(eq3_7); characteristic polynomials eq. (eqdp_1); the small-c expansion of
the physical eigenvalue, eq. (eqdp_2)-(eqdp_5); and the discrete symbol of
the median-dual operator on a consistently split rectangular torus, which
turns the mesh scheme into the scalar recursion of eq. (eq3_7).
"""
from __future__ import annotations

import numpy as np


# ---- split-explicit (dissipative forward-backward), eq. (eq3_6)/(eq3_7) -----
def se_matrix(c, theta):
    """Amplification matrix of eq. (eq3_7) acting on (eta~, u~)."""
    return np.array([[1.0 - c * c * (1.0 + theta), -1j * c], [-1j * c, 1.0]], dtype=complex)


def se_char_poly_coeffs(c, theta):
    """Coefficients (lambda^0, lambda^1, lambda^2) of P_SE in eq. (eqdp_1)."""
    return np.array([1.0 - c * c * theta, c * c * theta + c * c - 2.0, 1.0])


def se_eigs(c, theta):
    c0, c1, c2 = se_char_poly_coeffs(c, theta)
    return np.roots([c2, c1, c0])


def se_physical_root(c, theta):
    """The eigenvalue that tends to exp(+ic) as c -> 0."""
    r = se_eigs(c, theta)
    return r[np.argmin(np.abs(r - np.exp(1j * c)))]


def se_expansion(theta):
    """(m, n, q) of lambda = 1 + m c + n c^2 + q c^3, eq. (eqdp_5); m = i."""
    return 1j, -0.5 * (1.0 + theta), -1j / 8.0 * (1.0 + theta) ** 2


def se_chi(theta):
    """Dissipation parameter, eq. (eqdp_4): 2 chi = theta."""
    return 0.5 * theta


def se_stability_limit(theta):
    """Largest c with |lambda| <= 1: c^2 (1 + 2 theta) <= 4."""
    return 2.0 / np.sqrt(1.0 + 2.0 * theta)


def per_step_response(c_baroclinic, M, theta):
    """Amplitude and phase error of the physical mode after M substeps of c/M."""
    lam = se_physical_root(c_baroclinic / M, theta)
    amp = abs(lam) ** M
    phase = M * np.angle(lam) - c_baroclinic
    return amp, phase


# ---- semi-implicit, eq. (eq3_3) ----------------------------------------------
def si_matrix(c, theta, alpha):
    k = 1.0 / (alpha * theta * c * c + 1.0)
    return k * np.array([[alpha * theta * c * c - alpha * c * c + 1.0, -1j * c],
                         [-1j * c, alpha * theta * c * c - theta * c * c + 1.0]], dtype=complex)


def si_char_poly_coeffs(c, theta, alpha):
    den = alpha * c * c * theta + 1.0
    c0 = (alpha * c * c * theta - alpha * c * c - c * c * theta + c * c + 1.0) / den
    c1 = (-2.0 * alpha * c * c * theta + alpha * c * c + c * c * theta - 2.0) / den
    return np.array([c0, c1, 1.0])


# ---- AB3-AM4 (SESM), eq. (eq3_5) ---------------------------------------------
def sesm_matrix(c, beta, delta, gamma, zeta):
    ic = 1j * c
    return np.array([
        [1, 0, 0, -ic * (1.5 + beta), ic * (0.5 + 2 * beta), -ic * beta],
        [1, 0, 0, 0, 0, 0],
        [0, 1, 0, 0, 0, 0],
        [-ic * (1 - gamma - zeta), -ic * gamma, -ic * zeta, 1 - c * c * delta * (1.5 + beta),
         c * c * delta * (0.5 + 2 * beta), -c * c * delta * beta],
        [0, 0, 0, 1, 0, 0],
        [0, 0, 0, 0, 1, 0]], dtype=complex)


def sesm_char_poly_coeffs(c, b, d, g, z):
    """lambda^0..lambda^6 of P_SESM in eq. (eqdp_1); the printed '+-' read as '-'."""
    c2 = c * c
    return np.array([
        b * z * c2,
        c2 * (b * (g - 2 * z) - z / 2),
        -c2 * ((d + 3 * g - 1) * b + g / 2 - 1.5 * z),
        c2 / 2 * (b * (6 * d + 6 * g + 4 * z - 4) + d + 4 * g + z - 1),
        1 + c2 / 2 * (b * (-6 * d - 2 * g - 2 * z + 2) - 4 * d - 3 * g - 3 * z + 3),
        -2 + c2 * d / 2 * (2 * b + 3),
        1.0])


def sesm_params(theta, beta=0.281105):
    """(beta, delta, gamma, zeta) of the SESM scheme at the dissipation of SE(theta).

    2 chi = theta (eq. (eqdp_4), SE line); beta of the largest stability limit
    (Sec. 3.2); zeta and gamma from eq. (eqdp_6), second line (no O(c^3) phase
    constraint; the setting of Fig. 2); delta from 2 chi = delta - gamma - 2 zeta - 1/2
    (eq. (eqdp_4), SESM line).
    """
    chi = 0.5 * theta
    zeta = 0.010 - 0.135 * chi
    gamma = 0.083 - 0.514 * chi
    delta = 2.0 * chi + gamma + 2.0 * zeta + 0.5
    return beta, delta, gamma, zeta


def sesm_stability_limit(beta, delta, gamma, zeta, c_max=3.0, n=3000):
    """Largest c on a grid below which every eigenvalue of eq. (eq3_5) has |lambda| <= 1."""
    last = 0.0
    for c in np.linspace(c_max / n, c_max, n):
        if np.max(np.abs(np.linalg.eigvals(sesm_matrix(c, beta, delta, gamma, zeta)))) > 1 + 1e-12:
            return last
        last = c
    return last


def sesm_torus_mode_amplitudes(c2, params, nsub, restart_every=None):
    """a_m: eta^m = a_m cos(k.x) from eta^0 = cos(k.x), U^0 = 0 under eq. (eq3_5).

    The history levels start equal to the initial state; with restart_every = n
    they are reset to the current state every n substeps (a new subcycle).
    """
    c = np.sqrt(c2)
    Mc = sesm_matrix(c, *params)
    v = np.array([1, 1, 1, 0, 0, 0], dtype=complex)
    out = [1.0]
    for m in range(1, nsub + 1):
        v = Mc @ v
        out.append(v[0])
        if restart_every and m % restart_every == 0:
            v = np.array([v[0], v[0], v[0], v[3], v[3], v[3]])
    out = np.array(out)
    assert np.max(np.abs(out.imag)) < 1e-12 * max(1.0, np.max(np.abs(out.real)))
    return out.real


# ---- mesh symbol on a consistently split rectangular torus --------------------
def torus_symbol(kx, ky, dx, dy):
    """Eigenvalue of -D G for exp(i k.x): the 5-point Laplacian symbol."""
    return (4.0 / dx ** 2) * np.sin(0.5 * kx * dx) ** 2 + (4.0 / dy ** 2) * np.sin(0.5 * ky * dy) ** 2


def torus_mode_amplitudes(c2, theta, nsub):
    """a_m, m = 0..nsub: eta^m = a_m cos(k.x) from eta^0 = cos(k.x), U^0 = 0.

    With psi = dt_s D U the mesh scheme reduces, mode by mode, to eq. (eq3_7)
    with u~ = psi / (i c); a_m is the first component of M_c^m (1, 0)^T.
    """
    c = np.sqrt(c2)
    Mc = se_matrix(c, theta)
    v = np.array([1.0 + 0j, 0.0 + 0j])
    out = [1.0]
    for _ in range(nsub):
        v = Mc @ v
        out.append(v[0])
    out = np.array(out)
    assert np.max(np.abs(out.imag)) < 1e-12 * max(1.0, np.max(np.abs(out.real)))
    return out.real
