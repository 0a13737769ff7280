"""Pins of the oracle's tangent-linear and adjoint models.

The TLM is pinned by central finite differences of the forward oracle; the
adjoint by the dot-product identity <lam, TLM(d)> = <ADJ(lam), d> and, on a
tiny mesh, by the full Jacobian assembled from finite differences.
"""
import numpy as np
import pytest

import oracle
import sesynth


def _case(kind, seed, linear_h=False, nsub=10):
    case = sesynth.random_case(sesynth.tiny_mesh(kind), seed=seed, linear_h=linear_h, nsub=nsub)
    return case, oracle.Mesh(case, reordered=False)


def _fwd(m, case, eta0, U0, R, H0):
    eta, U, Uavg, _ = m.subcycle(eta0, U0, H0=H0, f=case["f"], R=R, g=case["g"],
                                 theta=case["theta"], nsub=case["nsub"], tau=case["tau"],
                                 linear_h=case["linear_h"], volume=False)
    return np.concatenate([eta, U.ravel(), Uavg.ravel()])


def _dirs(case, seed):
    r = sesynth.rng(seed)
    nv, ne = case["H0"].size, case["f"].size
    return (r.standard_normal(nv) * 0.1, r.standard_normal((ne, 2)) * 10.0,
            r.standard_normal((ne, 2)) * 0.01, r.standard_normal(nv) * 50.0)


@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86"])
@pytest.mark.parametrize("linear_h", [False, True])
def test_tlm_matches_central_differences(kind, linear_h):
    case, m = _case(kind, 21, linear_h)
    d_eta, d_U, d_R, d_H0 = _dirs(case, 22)
    x = (case["eta0"], case["U0"], case["R"], case["H0"])
    tl = m.tlm(case["eta0"], case["U0"], d_eta, d_U, d_R, d_H0, H0=case["H0"], f=case["f"],
               R=case["R"], g=case["g"], theta=case["theta"], nsub=case["nsub"],
               tau=case["tau"], linear_h=linear_h)
    tl = np.concatenate([tl[0], tl[1].ravel(), tl[2].ravel()])
    h = 1e-4
    plus = _fwd(m, case, *(xi + h * di for xi, di in zip(x, (d_eta, d_U, d_R, d_H0))))
    minus = _fwd(m, case, *(xi - h * di for xi, di in zip(x, (d_eta, d_U, d_R, d_H0))))
    fd = (plus - minus) / (2 * h)
    assert np.max(np.abs(fd - tl)) <= 1e-6 * np.max(np.abs(tl))


@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86"])
@pytest.mark.parametrize("linear_h", [False, True])
def test_adjoint_dot_product(kind, linear_h):
    case, m = _case(kind, 31, linear_h, nsub=17)
    nv, ne = case["H0"].size, case["f"].size
    d_eta, d_U, d_R, d_H0 = _dirs(case, 32)
    r = sesynth.rng(33)
    l_eta, l_U, l_Ua = r.standard_normal(nv), r.standard_normal((ne, 2)), r.standard_normal((ne, 2))
    kw = dict(H0=case["H0"], f=case["f"], R=case["R"], g=case["g"], theta=case["theta"],
              nsub=case["nsub"], tau=case["tau"], linear_h=linear_h)
    te, tU, tUa = m.tlm(case["eta0"], case["U0"], d_eta, d_U, d_R, d_H0, **kw)
    ge, gU, gR, gH = m.adjoint(case["eta0"], case["U0"], l_eta, l_U, l_Ua, **kw)
    lhs = np.sum(l_eta * te) + np.sum(l_U * tU) + np.sum(l_Ua * tUa)
    rhs = np.sum(ge * d_eta) + np.sum(gU * d_U) + np.sum(gR * d_R) + np.sum(gH * d_H0)
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1e-300) * 10


def test_adjoint_equals_jacobian_transpose():
    """Every column of the FD Jacobian of eta^M w.r.t. (eta0, H0) against the adjoint rows."""
    case, m = _case("grid3", 41, False, nsub=6)
    nv = case["H0"].size
    r = sesynth.rng(42)
    lam = r.standard_normal(nv)
    kw = dict(H0=case["H0"], f=case["f"], R=case["R"], g=case["g"], theta=case["theta"],
              nsub=case["nsub"], tau=case["tau"])
    ge, gU, gR, gH = m.adjoint(case["eta0"], case["U0"], lam, None, None, **kw)
    h = 1e-5
    for j in range(nv):
        e = np.zeros(nv)
        e[j] = 1.0
        fp = m.subcycle(case["eta0"] + h * e, case["U0"], **kw)[0]
        fm = m.subcycle(case["eta0"] - h * e, case["U0"], **kw)[0]
        assert abs(np.dot(lam, (fp - fm) / (2 * h)) - ge[j]) <= 1e-7 * np.abs(ge).max()
        kw2 = dict(kw)
        kw2["H0"] = case["H0"] + 100 * h * e
        fp = m.subcycle(case["eta0"], case["U0"], **kw2)[0]
        kw2["H0"] = case["H0"] - 100 * h * e
        fm = m.subcycle(case["eta0"], case["U0"], **kw2)[0]
        assert abs(np.dot(lam, (fp - fm) / (200 * h)) - gH[j]) <= 1e-6 * np.abs(gH).max()


def test_adjoint_area_weighted_loss_fd():
    """Loss sum_v A_v (eta^M - target)^2 (the adjoint workload): gradient vs FD."""
    case, m = _case("jitter76", 51, False, nsub=12)
    r = sesynth.rng(52)
    target = 0.3 * r.standard_normal(case["H0"].size)
    kw = dict(H0=case["H0"], f=case["f"], R=case["R"], g=case["g"], theta=case["theta"],
              nsub=case["nsub"], tau=case["tau"])

    def loss(eta0, U0, R, H0):
        k = dict(kw, R=R, H0=H0)
        eta = m.subcycle(eta0, U0, **k)[0]
        return np.sum(m.Av * (eta - target) ** 2)

    etaM = m.subcycle(case["eta0"], case["U0"], **kw)[0]
    ge, gU, gR, gH = m.adjoint(case["eta0"], case["U0"], 2 * m.Av * (etaM - target), **kw)
    x = [case["eta0"], case["U0"], case["R"], case["H0"]]
    grads = [ge, gU, gR, gH]
    for i in range(4):
        d = r.standard_normal(x[i].shape)
        h = 1e-6 * np.abs(x[i]).max()
        xp = list(x)
        xm = list(x)
        xp[i] = x[i] + h * d
        xm[i] = x[i] - h * d
        fd = (loss(*xp) - loss(*xm)) / (2 * h)
        an = np.sum(grads[i] * d)
        assert abs(fd - an) <= 1e-6 * abs(an)
