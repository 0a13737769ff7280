"""Pins of the oracle's barotropic viscous regularization, eq. (eq:viscosity_BT),
R^hV = div(H A grad(U / H)), and of the subcycle that carries it.

What fixes the operator independently of the oracle's code:
  * convergence to the continuous operator: on equilateral tori of side s, with
    A = A0 constant, the discrete term approaches A0 (d_xx + d_yy) U for constant H
    and div(H A0 grad u) for depth varying across the flow, with the error
    shrinking with s (a wrong factor anywhere converges to another limit);
  * the edge-by-edge construction of oracle/brute.py (interior edges from a
    dictionary of vertex pairs, scatter of each flux to both triangles, centroid
    distance from the opposite vertices, shoelace areas);
  * summation by parts: sum_e A_e u_e . V_e equals minus the sum over interior
    edges of H A (l/d) |du|^2 (so the term dissipates), sum_e A_e V_e vanishes,
    and a uniform velocity gives zero;
  * the subcycle: zero coefficients reproduce the plain subcycle bit for bit,
    the lake at rest stays exact, and the dense brute-force subcycle with the
    viscous term agrees.
"""
import numpy as np
import pytest

import oracle
import sesynth
from oracle import brute

KINDS = ["jitter76", "chan54", "sphere86", "torus43"]


def _case(kind, seed=3):
    return sesynth.random_case(sesynth.tiny_mesh(kind), seed=seed, nsub=16)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("A0,Cv,linear_h", [(300.0, 0.0, False), (50.0, 0.2, False),
                                            (0.0, 0.5, True)])
def test_operator_matches_edge_construction(kind, A0, Cv, linear_h):
    c = _case(kind)
    m = oracle.Mesh(c, reordered=False)
    V = m.visc(c["eta0"], c["U0"], H0=c["H0"], A0=A0, Cv=Cv, linear_h=linear_h)
    Vb, energy = brute.visc_operator(c, c["eta0"], c["U0"], H0=c["H0"], A0=A0, Cv=Cv,
                                     linear_h=linear_h, return_energy=True)
    assert np.abs(V - Vb).max() <= 1e-12 * np.abs(Vb).max()
    # summation by parts: the term removes kinetic energy, edge by edge
    Hv = c["H0"] if linear_h else c["H0"] + c["eta0"]
    u = c["U0"] / Hv[c["tri"]].mean(axis=1)[:, None]
    work = np.sum(m.Ae[:, None] * u * V)
    assert energy < 0 and abs(work - energy) <= 1e-12 * abs(energy)
    # conservation: fluxes cancel in pairs
    flux_scale = np.abs(m.Ae[:, None] * V).sum()
    assert np.abs((m.Ae[:, None] * V).sum(axis=0)).max() <= 1e-13 * flux_scale


@pytest.mark.parametrize("kind", KINDS)
def test_uniform_velocity_gives_zero(kind):
    c = _case(kind, seed=5)
    m = oracle.Mesh(c, reordered=False)
    He = (c["H0"] + c["eta0"])[c["tri"]].mean(axis=1)
    U = np.outer(He, [0.3, -0.2])
    V = m.visc(c["eta0"], U, H0=c["H0"], A0=500.0, Cv=0.3)
    # u = U/H_e = (0.3, -0.2) to rounding; the fluxes are rounding-sized
    scale = 500.0 * c["H0"].max() * 0.3 / m.Ae.min() * 4.0
    assert np.abs(V).max() <= 1e-13 * scale


def _torus_fields(n, s, kx_modes, ky_modes):
    t = sesynth.equilateral_torus(n, s)
    m = oracle.Mesh(t, reordered=False)
    X = t["x"][t["tri"]]
    Y = t["y"][t["tri"]]
    # triangle centroids: unwrap x around the first vertex
    Px = t["period_x"]
    dX = (X - X[:, :1] + Px / 2) % Px - Px / 2
    cx = X[:, 0] + dX.mean(axis=1)
    Py = t["period_y"]
    dY = (Y - Y[:, :1] + Py / 2) % Py - Py / 2
    cy = Y[:, 0] + dY.mean(axis=1)
    kx = 2 * np.pi * kx_modes / Px
    ky = 2 * np.pi * ky_modes / Py
    return t, m, cx, cy, kx, ky


def test_converges_to_the_laplacian_for_constant_depth():
    A0, H = 250.0, 4000.0
    errs = []
    for n in (12, 24, 48):
        s = 96e3 / n
        t, m, cx, cy, kx, ky = _torus_fields(n, s, 1, 1)
        phase = kx * cx + ky * cy
        U = np.stack([np.cos(phase), 0.5 * np.sin(phase)], -1) * H
        V = m.visc(np.zeros(t["x"].size), U, H0=t["H0"], A0=A0, Cv=0.0, linear_h=True)
        exact = -A0 * (kx ** 2 + ky ** 2) * U
        errs.append(np.abs(V - exact).max() / np.abs(exact).max())
    assert errs[2] < 0.1
    assert errs[1] / errs[0] < 0.6 and errs[2] / errs[1] < 0.6, errs


def test_converges_with_depth_varying_across_the_flow():
    """u = (cos(k y), 0), H = H0 (1 + 0.3 cos(k x)): div(H A0 grad u) = -A0 k^2 H(x) cos(k y)."""
    A0, H0 = 250.0, 4000.0
    errs = []
    for n in (12, 24, 48):
        s = 96e3 / n
        t, m, cx, cy, kx, ky = _torus_fields(n, s, 1, 1)
        Hv = H0 * (1.0 + 0.3 * np.cos(kx * t["x"]))
        He = Hv[t["tri"]].mean(axis=1)
        U = np.stack([He * np.cos(ky * cy), np.zeros_like(cy)], -1)
        V = m.visc(np.zeros(t["x"].size), U, H0=Hv, A0=A0, Cv=0.0, linear_h=True)
        exact = -A0 * ky ** 2 * H0 * (1.0 + 0.3 * np.cos(kx * cx)) * np.cos(ky * cy)
        errs.append(np.abs(V[:, 0] - exact).max() / np.abs(exact).max())
        assert np.abs(V[:, 1]).max() <= 0.2 * np.abs(exact).max()
    assert errs[2] < 0.1
    assert errs[1] / errs[0] < 0.6 and errs[2] / errs[1] < 0.6, errs


def _sub(m, c, visc, nsub=None, **kw):
    args = dict(H0=c["H0"], f=c["f"], R=c["R"], g=c["g"], theta=c["theta"],
                nsub=nsub or c["nsub"], tau=c["tau"], linear_h=c["linear_h"])
    args.update(kw)
    return m.subcycle(c["eta0"], c["U0"], visc=visc, **args)


def test_zero_coefficients_reproduce_the_plain_subcycle():
    c = _case("jitter76")
    m = oracle.Mesh(c, reordered=False)
    a = _sub(m, c, None)
    b = _sub(m, c, (0.0, 0.0))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("kind", KINDS)
def test_viscous_subcycle_matches_dense_brute_force(kind):
    c = _case(kind, seed=7)
    m = oracle.Mesh(c, reordered=False)
    # background coefficient at a fixed fraction of the explicit limit ~ A_e / dt_s
    visc = (0.02 * m.Ae.mean() * c["nsub"] / c["tau"], 0.5)
    eta, U, Uavg, _ = _sub(m, c, visc)
    ops = brute.dense_operators(c)
    e2, U2, A2 = brute.subcycle(ops, c["eta0"], c["U0"], H0=c["H0"], f=c["f"], R=c["R"],
                                g=c["g"], theta=c["theta"], nsub=c["nsub"], tau=c["tau"],
                                linear_h=c["linear_h"], visc=visc, mesh=c)
    assert np.abs(eta - e2).max() <= 1e-11 * np.abs(c["eta0"]).max()
    assert np.abs(U - U2).max() <= 1e-11 * np.abs(c["U0"]).max()
    assert np.abs(Uavg - A2).max() <= 1e-11 * np.abs(c["U0"]).max()
    # the term matters at this strength: without it the result differs
    e3 = _sub(m, c, None)[0]
    assert np.abs(e3 - eta).max() > 1e3 * 1e-11 * np.abs(c["eta0"]).max()


def test_viscous_lake_at_rest_exact():
    c = _case("sphere86")
    c["eta0"] = np.full_like(c["eta0"], 0.5)
    c["U0"] = np.zeros_like(c["U0"])
    c["R"] = np.zeros_like(c["R"])
    m = oracle.Mesh(c, reordered=False)
    eta, U, Uavg, _ = _sub(m, c, (1000.0, 0.5))
    assert np.all(eta == 0.5) and np.all(U == 0.0) and np.all(Uavg == 0.0)


def test_neighbour_table_is_symmetric():
    for kind in KINDS:
        c = sesynth.tiny_mesh(kind)
        m = oracle.Mesh(c, reordered=True)
        nb, l, lod = m.visc_geometry()
        for e in range(m.ne):
            for j in range(3):
                n = nb[e, j]
                if n < 0:
                    assert l[e, j] == 0.0
                    continue
                back = np.nonzero(nb[n] == e)[0]
                assert back.size == 1
                jb = back[0]
                assert {m.tri[e, j], m.tri[e, (j + 1) % 3]} == {m.tri[n, jb], m.tri[n, (jb + 1) % 3]}
                assert abs(l[e, j] - l[n, jb]) <= 1e-12 * l[e, j]
                assert abs(lod[e, j] - lod[n, jb]) <= 1e-12 * lod[e, j]
