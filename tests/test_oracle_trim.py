"""Pins of the oracle's consumer of the averaged transport: the trim of the
layer transports (eq. (eq4_13)), the z* thickness target (Sec. 2.4) and the
diasurface velocity from the thickness equation.

What fixes it: the trimmed transports sum to <<U>> (eq. (eq4_13)); the z*
thicknesses sum to H0 + eta^{n+1}; with eta^{n+1} and <<U>> from a real
subcycle the surface diasurface velocity vanishes to rounding (column volume
closure, eqs. (eq4_11)-(eq4_13)) and does not with a wrong transport; an
independent dense divergence (oracle/brute.py) reproduces every output.
"""
import numpy as np
import pytest

import oracle
import sesynth
from oracle import brute


def _setup(kind="jitter76", K=12, seed=2, W=None):
    mesh = sesynth.tiny_mesh(kind)
    case = sesynth.random_case(mesh, seed=seed, nsub=24)
    m = oracle.Mesh(case, reordered=False)
    eta1, U1, Uavg, _ = m.subcycle(case["eta0"], case["U0"], H0=case["H0"], f=case["f"],
                                   R=case["R"], W=W, g=case["g"], theta=case["theta"],
                                   nsub=case["nsub"], tau=case["tau"])
    lay = sesynth.layers(case, K=K, seed=seed)
    h0 = case["H0"][:, None] * lay["frac"][None, :]
    hn = h0 * ((case["H0"] + case["eta0"]) / case["H0"])[:, None]
    return case, m, eta1, Uavg, lay, h0, hn


@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86"])
@pytest.mark.parametrize("with_w", [False, True])
def test_trim_sums_zstar_and_column_closure(kind, with_w):
    mesh = sesynth.tiny_mesh(kind)
    W = 2e-5 * sesynth.rng(8).standard_normal(mesh["x"].size) if with_w else None
    case, m, eta1, Uavg, lay, h0, hn = _setup(kind, W=W)
    U, hnew, w = m.trim_zstar(H0=case["H0"], eta_new=eta1, Uavg=Uavg, Ustar=lay["Ustar"], hn=hn,
                              h0=h0, W=W, tau=case["tau"])
    # eq. (eq4_13): the trimmed layers carry the averaged transport
    assert np.max(np.abs(U.sum(axis=1) - Uavg)) <= 1e-12 * np.abs(Uavg).max()
    # z*: common stretching, column thickness H0 + eta^{n+1}
    ratio = hnew / h0
    assert np.max(np.abs(ratio - ratio[:, :1])) <= 1e-14
    assert np.max(np.abs(hnew.sum(1) - (case["H0"] + eta1))) <= 1e-12 * case["H0"].max()
    # bottom boundary and column closure at the surface
    assert np.all(w[:, -1] == 0.0)
    # rounding of the thickness change: relative 1e-12 of the column over tau
    assert np.max(np.abs(w[:, 0])) <= 1e-12 * case["H0"].max() / case["tau"]


def test_surface_residual_detects_a_wrong_transport():
    case, m, eta1, Uavg, lay, h0, hn = _setup()
    bad = Uavg * 1.001
    _, _, w = m.trim_zstar(H0=case["H0"], eta_new=eta1, Uavg=bad, Ustar=lay["Ustar"], hn=hn,
                           h0=h0, tau=case["tau"])
    assert np.max(np.abs(w[:, 0])) > 1e3 * 1e-12 * case["H0"].max() / case["tau"]


def test_trim_matches_dense_construction():
    W = 1e-5 * sesynth.rng(3).standard_normal(sesynth.tiny_mesh("chan54")["x"].size)
    case, m, eta1, Uavg, lay, h0, hn = _setup("chan54", K=7, W=W)
    U, hnew, w = m.trim_zstar(H0=case["H0"], eta_new=eta1, Uavg=Uavg, Ustar=lay["Ustar"], hn=hn,
                              h0=h0, W=W, tau=case["tau"])
    ops = brute.dense_operators(case)
    tri = np.asarray(case["tri"])
    K = lay["K"]
    hn1 = h0 * ((case["H0"] + eta1) / case["H0"])[:, None]
    hmid = 0.5 * (hn + hn1)
    he = ops["P"] @ hmid                              # triangle means [ne][K]
    Us = lay["Ustar"]
    Ut = Us - (he / he.sum(1, keepdims=True))[:, :, None] * (Us.sum(1) - Uavg)[:, None, :]
    div = np.stack([ops["D"] @ Ut[:, k, :].reshape(-1) for k in range(K)], axis=1)
    wb = np.zeros((tri.max() + 1, K + 1))
    for k in range(K - 1, -1, -1):
        wb[:, k] = wb[:, k + 1] - (hn1[:, k] - hn[:, k]) / case["tau"] - div[:, k] \
            - (W if k == 0 else 0.0)
    assert np.max(np.abs(hnew - hn1)) <= 1e-12 * hn1.max()
    assert np.max(np.abs(U - Ut)) <= 1e-12 * np.abs(Ut).max()
    assert np.max(np.abs(w - wb)) <= 1e-10 * np.abs(wb).max()


def test_trim_is_identity_when_layers_already_sum_to_the_average():
    case, m, eta1, Uavg, lay, h0, hn = _setup()
    Us = lay["Ustar"].copy()
    Us[:, -1, :] += Uavg - Us.sum(1)
    U, _, _ = m.trim_zstar(H0=case["H0"], eta_new=eta1, Uavg=Uavg, Ustar=Us, hn=hn, h0=h0,
                           tau=case["tau"])
    assert np.max(np.abs(U - Us)) <= 1e-12 * np.abs(Us).max()


def test_lake_at_rest():
    case, m, eta1, Uavg, lay, h0, hn = _setup()
    z = np.zeros_like(case["eta0"])
    U, hnew, w = m.trim_zstar(H0=case["H0"], eta_new=z, Uavg=np.zeros_like(Uavg),
                              Ustar=np.zeros_like(lay["Ustar"]), hn=h0, h0=h0, tau=case["tau"])
    assert np.all(U == 0.0) and np.all(hnew == h0) and np.all(w == 0.0)
