"""Pins of the FP64 oracle's AB3-AM4 (SESM) substep, eqs. (eq4_7)-(eq4_8).

What fixes the scheme:
  * on a consistently split torus (f = 0, linear H) the mesh scheme reduces,
    mode by mode, to the prototype recursion of eq. (eq3_5), whose matrix is
    printed in the paper (and pinned against eq. (eqdp_1) in
    test_oracle_analysis.py);
  * with a flat surface the transport follows the AB3 extrapolation of the
    inertial oscillation, whose solution the roots of its characteristic
    polynomial give;
  * the dense-operator construction of oracle/brute.py (independent geometry)
    reproduces it on random fields (nonlinear depth, Coriolis, forcing, W);
  * volume conservation, telescoping of the elevation over the subcycle, and
    the lake at rest hold to rounding.
"""
import numpy as np
import pytest

import oracle
import sesynth
from oracle import analytic, brute

G = 9.81
P = analytic.sesm_params(0.14)


def _sesm(m, case, eta=None, U=None, nsub=None, tau=None, W=None, params=P, **over):
    kw = dict(H0=case["H0"], f=case["f"], R=case["R"], W=W, g=case["g"], nsub=nsub or case["nsub"],
              tau=tau or case["tau"], linear_h=case["linear_h"])
    kw.update(over)
    b, d, gm, z = params
    return m.subcycle_sesm(case["eta0"] if eta is None else eta,
                           case["U0"] if U is None else U, beta=b, delta=d, gamma=gm, zeta=z,
                           **kw)


def test_sesm_parameters_at_chi_007():
    """eq. (eqdp_6) second line and eq. (eqdp_4) at chi = 0.07 (theta = 0.14)."""
    b, d, gm, z = analytic.sesm_params(0.14)
    assert b == 0.281105
    assert abs(z - 0.00055) < 1e-12 and abs(gm - 0.04702) < 1e-12
    assert abs(d - 0.68812) < 1e-12
    # the dissipation of eq. (eqdp_4): 2 chi = delta - gamma - 2 zeta - 1/2
    assert abs((d - gm - 2 * z - 0.5) - 0.14) < 1e-12


@pytest.mark.parametrize("px,py,dts", [(3, 2, 25.0), (1, 0, 30.0), (7, 5, 18.0), (10, 7, 20.0)])
def test_sesm_torus_mode_matches_eq3_5(px, py, dts):
    nx, ny, dx, dy = 32, 16, 10e3, 12e3
    H = 4000.0
    t = sesynth.torus(nx, ny, dx, dy, H=H)
    kx, ky = 2 * np.pi * px / (nx * dx), 2 * np.pi * py / (ny * dy)
    eta0 = np.cos(kx * t["x"] + ky * t["y"])
    c2 = G * H * dts ** 2 * analytic.torus_symbol(kx, ky, dx, dy)
    assert np.sqrt(c2) < analytic.sesm_stability_limit(*P)
    m = oracle.Mesh(t, reordered=False)
    n = 150
    a = analytic.sesm_torus_mode_amplitudes(c2, P, 3 * n, restart_every=n)
    eta, U = eta0, t["U0"]
    for chunk in range(3):           # 3 chained subcycles; histories restart each time
        eta, U, _, _ = _sesm(m, t, eta=eta, U=U, nsub=n, tau=n * dts)
        assert np.max(np.abs(eta - a[n * (chunk + 1)] * eta0)) <= 1e-12


def test_sesm_inertial_oscillation_follows_ab3_roots():
    """Flat surface, uniform transport, f const: w = U_x + i U_y obeys
    w^{m+1} = w^m - i f dt_s w_ab, solved through the roots of its polynomial."""
    t = sesynth.torus(8, 6, 10e3, 10e3, H=3000.0, f=1.1e-4, linear_h=False)
    m = oracle.Mesh(t, reordered=False)
    U0 = np.tile([0.7, -0.3], (t["tri"].shape[0], 1))
    eta0 = np.full(t["x"].size, 0.25)
    dts, nsub = 300.0, 40
    eta, U, Uavg, _ = _sesm(m, t, eta=eta0, U=U0, nsub=nsub, tau=nsub * dts)
    b = P[0]
    h = 1j * 1.1e-4 * dts
    # r^3 = r^2 - h ((3/2 + b) r^2 - (1/2 + 2b) r + b)
    coef = [1.0, -(1.0 - h * (1.5 + b)), -h * (0.5 + 2 * b), h * b]
    r = np.roots(coef)
    w0 = 0.7 - 0.3j
    # w^{-2} = w^{-1} = w^0 = w0 fix the three constants
    V = np.array([[rr ** k for rr in r] for k in (-2, -1, 0)])
    cst = np.linalg.solve(V, np.full(3, w0))
    wM = np.sum(cst * r ** nsub)
    assert np.max(np.abs(U[:, 0] - wM.real)) <= 1e-12 and np.max(np.abs(U[:, 1] - wM.imag)) <= 1e-12
    # the elevation stays flat: a uniform transport has no divergence on the torus
    assert np.max(np.abs(eta - 0.25)) <= 1e-13
    # averaged transport: mean of the AB3 transports
    wab = [(1.5 + b) * np.sum(cst * r ** k) - (0.5 + 2 * b) * np.sum(cst * r ** (k - 1))
           + b * np.sum(cst * r ** (k - 2)) for k in range(nsub)]
    wav = np.mean(wab)
    assert np.max(np.abs(Uavg[:, 0] - wav.real)) <= 1e-12
    assert np.max(np.abs(Uavg[:, 1] - wav.imag)) <= 1e-12


@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86", "torus43"])
@pytest.mark.parametrize("with_w", [False, True])
def test_sesm_matches_dense_operators(kind, with_w):
    mesh = sesynth.tiny_mesh(kind)
    case = sesynth.random_case(mesh, seed=5, nsub=24)
    W = 1e-4 * sesynth.rng(41).standard_normal(mesh["x"].size) if with_w else None
    m = oracle.Mesh(case, reordered=False)
    eta, U, Uavg, _ = _sesm(m, case, W=W)
    ops = brute.dense_operators(case)
    b, d, gm, z = P
    e2, U2, A2 = brute.subcycle_sesm(ops, case["eta0"], case["U0"], H0=case["H0"], f=case["f"],
                                     R=case["R"], W=W, g=case["g"], beta=b, delta=d, gamma=gm,
                                     zeta=z, nsub=case["nsub"], tau=case["tau"])
    assert np.max(np.abs(eta - e2)) <= 1e-11 * np.abs(case["eta0"]).max()
    assert np.max(np.abs(U - U2)) <= 1e-11 * np.abs(case["U0"]).max()
    assert np.max(np.abs(Uavg - A2)) <= 1e-11 * np.abs(case["U0"]).max()


def test_sesm_volume_conserved_and_elevation_telescopes():
    """Sec. 2.4: no coastline flux, W = 0 -> sum_v A_v eta_v is constant; the
    summed elevation equation gives eta^M - eta^0 = -tau D <<U>> (the mean AB3
    transport), the counterpart of eq. (eq4_11)."""
    mesh = sesynth.tiny_mesh("jitter76")
    case = sesynth.random_case(mesh, seed=9, nsub=30, tau=30.0)
    m = oracle.Mesh(case, reordered=False)
    eta, U, Uavg, vol = _sesm(m, case)
    atot = m.Av.sum()
    assert np.max(np.abs(vol - vol[0])) <= 1e-13 * atot * np.abs(case["eta0"]).max()
    ops = brute.dense_operators(case)
    r = eta - case["eta0"] + case["tau"] * (ops["D"] @ Uavg.reshape(-1))
    assert np.max(np.abs(r)) <= 1e-11 * np.abs(case["eta0"]).max()


@pytest.mark.parametrize("kind", ["jitter76", "sphere86"])
def test_sesm_lake_at_rest_exact(kind):
    mesh = sesynth.tiny_mesh(kind)
    case = sesynth.random_case(mesh, seed=3, nsub=24)
    case["eta0"] = np.full_like(case["eta0"], 0.5)
    case["U0"] = np.zeros_like(case["U0"])
    case["R"] = np.zeros_like(case["R"])
    m = oracle.Mesh(case, reordered=False)
    eta, U, Uavg, _ = _sesm(m, case)
    assert np.all(eta == 0.5) and np.all(U == 0.0) and np.all(Uavg == 0.0)


def test_sesm_mutations_are_caught():
    """Parameter slips that a reading error would produce change the result beyond
    the tolerance of the dense check (guards the strength of that pin)."""
    mesh = sesynth.tiny_mesh("jitter76")
    case = sesynth.random_case(mesh, seed=5, nsub=24)
    m = oracle.Mesh(case, reordered=False)
    ref = _sesm(m, case)[0]
    b, d, gm, z = P
    for bad in ((b, d, gm + 1e-3, z), (b, d, gm, z + 1e-3), (b + 1e-3, d, gm, z),
                (b, d + 1e-3, gm, z)):
        assert np.max(np.abs(_sesm(m, case, params=bad)[0] - ref)) > 1e-9
