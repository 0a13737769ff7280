"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the property it checks and the passage that fixes it.  A
plausible slip anywhere in the oracle (pressure sign, Coriolis sign, theta
placement, a dropped forcing term, a wrong basis gradient or area, the sum
range of the averaged transport) fails at least one of them.
"""
import numpy as np
import pytest

import oracle
import sesynth
from oracle import analytic, brute

G, TH = 9.81, 0.14


def _run(case, mesh=None, nsub=None, tau=None, W=None, **over):
    m = mesh or oracle.Mesh(case, reordered=False)
    kw = dict(H0=case["H0"], f=case["f"], R=case["R"], W=W, g=case["g"],
              theta=case["theta"], nsub=nsub or case["nsub"], tau=tau or case["tau"],
              linear_h=case["linear_h"])
    kw.update(over)
    return m, m.subcycle(case["eta0"], case["U0"], **kw)


# --------------------------------------------------------------------------
# Lake at rest (Sec. 2.2: with eta constant, U = 0, R = 0 and W = 0 the
# barotropic system has no force; the difference-form gradient is exactly 0)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("level", [0.0, 0.5])
@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86"])
def test_lake_at_rest_exact(level, kind):
    mesh = sesynth.tiny_mesh(kind)
    case = sesynth.random_case(mesh, seed=3)
    case["eta0"] = np.full_like(case["eta0"], level)
    case["U0"] = np.zeros_like(case["U0"])
    case["R"] = np.zeros_like(case["R"])
    _, (eta, U, Uavg, vol) = _run(case, nsub=50)
    assert np.all(eta == level)
    assert np.all(U == 0.0) and np.all(Uavg == 0.0)


def test_lake_at_rest_c1_scale():
    case = sesynth.basin_c1()
    r = sesynth.rng(11)
    case["H0"] = r.uniform(100.0, 5000.0, case["H0"].size)
    case["eta0"] = np.full_like(case["eta0"], 0.37)
    m, (eta, U, Uavg, vol) = _run(case, nsub=30)
    assert np.all(eta == 0.37) and np.all(U == 0.0)


# --------------------------------------------------------------------------
# Volume conservation (Sec. 2.4: the averaged transport conserves volume;
# with no coastline flux the elevation equation conserves sum_v A_v eta_v)
# --------------------------------------------------------------------------
def test_volume_conservation_c1():
    case = sesynth.basin_c1()
    res = oracle.run_case(case)
    v = res["volume"]
    atot = res["mesh"].Av.sum()
    assert v.size == case["nsub"] * case["nsteps"] + 1
    assert np.max(np.abs(v - v[0])) <= 1e-13 * atot * np.abs(case["eta0"]).max()


@pytest.mark.parametrize("kind", ["jitter76", "sphere86"])
def test_volume_conservation_random(kind):
    case = sesynth.random_case(sesynth.tiny_mesh(kind), seed=5)
    m, (eta, U, Uavg, vol) = _run(case, nsub=600, tau=600 * 1.0)
    assert np.max(np.abs(vol - vol[0])) <= 1e-13 * m.Av.sum() * np.abs(case["eta0"]).max()


def test_volume_changes_with_freshwater_flux():
    """W enters the eta line (eq. (eq4_5)): V^M - V^0 = -tau sum_v A_v W_v."""
    case = sesynth.random_case(sesynth.tiny_mesh("jitter65"), seed=6)
    W = np.full(case["H0"].size, 1e-6)
    m, (eta, U, Uavg, vol) = _run(case, W=W)
    expect = -case["tau"] * np.sum(m.Av * W)
    assert abs((vol[-1] - vol[0]) - expect) <= 1e-10 * abs(expect)


# --------------------------------------------------------------------------
# Summed elevation equation, eq. (eq4_11)-(eq4_12): eta^M - eta^0 = -tau D <<U>>
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86"])
def test_telescoping_identity(kind):
    case = sesynth.random_case(sesynth.tiny_mesh(kind), seed=7)
    m, (eta, U, Uavg, vol) = _run(case)
    ops = brute.dense_operators(case)
    resid = eta - case["eta0"] + case["tau"] * (ops["D"] @ Uavg.reshape(-1))
    assert np.max(np.abs(resid)) <= 1e-12 * np.abs(case["eta0"]).max()


def test_telescoping_rejects_other_sum_ranges():
    """Only m = 1..M plus theta/M (U^M - U^0) closes eq. (eq4_11)."""
    case = sesynth.random_case(sesynth.tiny_mesh("jitter65"), seed=8)
    m = oracle.Mesh(case, reordered=False)
    ops = brute.dense_operators(case)
    eta, U = case["eta0"], case["U0"]
    Us = [U]
    M = case["nsub"]
    for _ in range(M):
        eta, U, _, _ = m.subcycle(eta, U, H0=case["H0"], f=case["f"], R=case["R"], g=G,
                                  theta=TH, nsub=1, tau=case["tau"] / M)
        Us.append(U)
    Us = np.array(Us)
    good = Us[1:].mean(0) + TH / M * (Us[-1] - Us[0])
    bad = Us[:-1].mean(0) + TH / M * (Us[-1] - Us[0])
    for avg, ok in ((good, True), (bad, False)):
        r = eta - case["eta0"] + case["tau"] * (ops["D"] @ avg.reshape(-1))
        assert (np.max(np.abs(r)) <= 1e-12 * np.abs(case["eta0"]).max()) == ok


# --------------------------------------------------------------------------
# Closed form on a consistently split torus: the mesh scheme reduces to the
# scalar recursion of eq. (eq3_7) with c^2 = g H dt_s^2 mu(k) (Sec. 3.1.3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("px,py,theta,dts", [(3, 2, 0.14, 30.0), (1, 0, 0.14, 33.0),
                                             (7, 5, 0.0, 20.0), (10, 7, 0.3, 25.0)])
def test_torus_mode_matches_eq3_7(px, py, theta, dts):
    nx, ny, dx, dy = 32, 16, 10e3, 12e3
    H = 4000.0
    t = sesynth.torus(nx, ny, dx, dy, H=H)
    kx, ky = 2 * np.pi * px / (nx * dx), 2 * np.pi * py / (ny * dy)
    eta0 = np.cos(kx * t["x"] + ky * t["y"])
    nsub = 600
    m = oracle.Mesh(t, reordered=False)
    c2 = G * H * dts ** 2 * analytic.torus_symbol(kx, ky, dx, dy)
    assert np.sqrt(c2) < analytic.se_stability_limit(theta)
    a = analytic.torus_mode_amplitudes(c2, theta, nsub)
    eta = eta0
    U = t["U0"]
    for chunk in range(6):           # 6 baroclinic steps of 100 substeps, chained
        eta, U, _, _ = m.subcycle(eta, U, H0=t["H0"], f=t["f"], R=t["R"], g=G, theta=theta,
                                  nsub=100, tau=100 * dts, linear_h=True)
        assert np.max(np.abs(eta - a[100 * (chunk + 1)] * eta0)) <= 1e-12


def test_torus_amplification_damping_and_phase_speed():
    """|lambda|^2 = 1 - theta c^2 (eq. (eqdp_1)); phase speed -> sqrt(g H) (eq. (eq3_1))."""
    nx, ny, dx, dy = 64, 8, 10e3, 10e3
    H, dts = 4000.0, 10.0
    t = sesynth.torus(nx, ny, dx, dy, H=H)
    m = oracle.Mesh(t, reordered=False)
    kx = 2 * np.pi / (nx * dx)
    eta0 = np.cos(kx * t["x"])
    probe = 0
    a = [1.0]
    eta, U = eta0, t["U0"]
    for _ in range(8):
        eta, U, _, _ = m.subcycle(eta, U, H0=t["H0"], f=t["f"], R=t["R"], g=G, theta=TH,
                                  nsub=1, tau=dts, linear_h=True)
        a.append(eta[probe] / eta0[probe])
    a = np.array(a)
    # a_{m+2} = tr a_{m+1} - det a_m  ->  least squares for (tr, det)
    A = np.column_stack([a[1:-1], -a[:-2]])
    tr, det = np.linalg.lstsq(A, a[2:], rcond=None)[0]
    c2 = G * H * dts ** 2 * analytic.torus_symbol(kx, 0.0, dx, dy)
    assert abs(det - (1 - TH * c2)) <= 1e-10
    assert abs(tr - (2 - (1 + TH) * c2)) <= 1e-10
    lam = np.roots([1.0, -tr, det])
    lam = lam[np.argmax(lam.imag)]
    speed = np.angle(lam) / (dts * kx)
    assert abs(speed / np.sqrt(G * H) - 1.0) < 2e-3


# --------------------------------------------------------------------------
# Spectrum of one substep on an arbitrary flat mesh (f = 0, linear H):
# eigenvalues = roots of P_SE(lambda; c_j), c_j^2 = g H dt_s^2 mu_j, plus the
# eigenvalue 1 of divergence-free transports (eq. (eqdp_1))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["jitter65", "chan54"])
def test_one_substep_spectrum(kind):
    mesh = sesynth.tiny_mesh(kind)
    nv, ne = mesh["x"].size, mesh["tri"].shape[0]
    H, dts = 3000.0, 2.0
    m = oracle.Mesh(mesh, reordered=False)
    n = nv + 2 * ne
    S = np.zeros((n, n))
    for j in range(n):
        z = np.zeros(n)
        z[j] = 1.0
        eta, U, _, _ = m.subcycle(z[:nv], z[nv:].reshape(ne, 2), H0=np.full(nv, H),
                                  f=np.zeros(ne), R=np.zeros((ne, 2)), g=G, theta=TH,
                                  nsub=1, tau=dts, linear_h=True)
        S[:nv, j] = eta
        S[nv:, j] = U.reshape(-1)
    ops = brute.dense_operators(mesh)
    mu = np.linalg.eigvals(-ops["D"] @ ops["G"]).real
    expect = [1.0] * (2 * ne - nv)
    for mj in mu:
        c = np.sqrt(max(G * H * dts ** 2 * mj, 0.0))
        if c < 1e-7:
            expect += [1.0, 1.0]
        else:
            expect += list(analytic.se_eigs(c, TH))
    got = np.linalg.eigvals(S)
    expect = np.array(expect, complex)
    # match as multisets
    used = np.zeros(expect.size, bool)
    worst = 0.0
    for lam in got:
        d = np.abs(expect - lam)
        d[used] = np.inf
        k = int(np.argmin(d))
        used[k] = True
        worst = max(worst, d[k])
    assert worst < 1e-6     # eigenvalue 1 is defective-free but clustered; see next line
    for lam in expect[np.abs(expect - 1.0) > 1e-3]:
        assert np.min(np.abs(got - lam)) < 1e-11


# --------------------------------------------------------------------------
# Coriolis: Crank-Nicolson rotation by -2 atan(f dt_s / 2) about the
# geostrophic point U* = (R_y, -R_x)/f (eq. (eq4_10), first line)
# --------------------------------------------------------------------------
def test_inertial_rotation_and_geostrophic_point():
    t = sesynth.torus(12, 10, 5e3, 6e3, H=2000.0, f=1.2e-3)
    nv, ne = t["x"].size, t["tri"].shape[0]
    R = np.tile([0.03, -0.05], (ne, 1))
    U0 = np.tile([1.5, -0.7], (ne, 1))
    eta0 = np.full(nv, 0.25)
    m = oracle.Mesh(t, reordered=False)
    dts, nsub = 10.0, 37
    r = sesynth.rng(4)
    eta, U, Uavg, _ = m.subcycle(eta0, U0, H0=r.uniform(500, 3000, nv), f=t["f"], R=R, g=G,
                                 theta=TH, nsub=nsub, tau=nsub * dts, linear_h=False)
    f = 1.2e-3
    Ustar = np.array([R[0, 1], -R[0, 0]]) / f
    ang = -2.0 * np.arctan(0.5 * f * dts) * nsub
    rot = np.array([[np.cos(ang), -np.sin(ang)], [np.sin(ang), np.cos(ang)]])
    expect = Ustar + rot @ (U0[0] - Ustar)
    assert np.max(np.abs(U - expect)) <= 1e-12 * np.abs(Ustar).max()
    assert np.max(np.abs(eta - 0.25)) <= 1e-15


# --------------------------------------------------------------------------
# Brute force: dense operators from an independent geometric construction
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["two", "grid3", "torus43", "jitter65", "jitter76", "chan54",
                                  "sphere86"])
@pytest.mark.parametrize("linear_h", [False, True])
def test_brute_force_all_terms(kind, linear_h):
    mesh = sesynth.tiny_mesh(kind)
    case = sesynth.random_case(mesh, seed=9, linear_h=linear_h)
    if kind == "sphere86":
        case["tau"], case["nsub"] = 240.0, 8
    r = sesynth.rng(10)
    W = 1e-5 * r.standard_normal(case["H0"].size)
    m, (eta, U, Uavg, _) = _run(case, W=W)
    ops = brute.dense_operators(case)
    eb, Ub, Uab = brute.subcycle(ops, case["eta0"], case["U0"], H0=case["H0"], f=case["f"],
                                 R=case["R"], W=W, g=G, theta=TH, nsub=case["nsub"],
                                 tau=case["tau"], linear_h=linear_h)
    assert np.max(np.abs(eta - eb)) <= 1e-13 * np.abs(eb).max()
    assert np.max(np.abs(U - Ub)) <= 1e-13 * np.abs(Ub).max()
    assert np.max(np.abs(Uavg - Uab)) <= 1e-13 * np.abs(Uab).max()
    assert np.max(np.abs(m.Av - ops["Av"])) <= 1e-14 * ops["Av"].max()
    assert np.max(np.abs(m.Ae - ops["Ae"])) <= 1e-14 * ops["Ae"].max()


def test_median_dual_areas_partition_the_domain():
    mesh = sesynth.tiny_mesh("jitter76")
    m = oracle.Mesh(mesh, reordered=False)
    assert abs(m.Av.sum() - m.Ae.sum()) <= 1e-12 * m.Ae.sum()
    # closed rectangle: total area equals the bounding box minus the jittered walls
    ops = brute.dense_operators(mesh)
    assert abs(ops["Av"].sum() - m.Ae.sum()) <= 1e-12 * m.Ae.sum()


def test_discrete_divergence_is_minus_adjoint_of_gradient():
    """<U, G eta>_{A_e} = -<D U, eta>_{A_v} (median-dual / P1 duality)."""
    mesh = sesynth.tiny_mesh("jitter76")
    ops = brute.dense_operators(mesh)
    r = sesynth.rng(12)
    eta = r.standard_normal(ops["nv"])
    U = r.standard_normal(2 * ops["ne"])
    lhs = np.sum(np.repeat(ops["Ae"], 2) * U * (ops["G"] @ eta))
    rhs = -np.sum(ops["Av"] * (ops["D"] @ U) * eta)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
