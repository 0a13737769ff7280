"""Pins of the oracle's vertically integrated baroclinic forcing, eq. (eq4_4).

What fixes it independently of the oracle's code:
  * a column worked by hand (tests/golden/forcing_column.txt);
  * the per-layer form of eq. (eq4_4): a column whose vertical-viscous tendencies
    are built layer by layer from interface stresses (surface stress on top,
    quadratic drag at the bottom, A_v du/dz between layers) and summed exactly
    with math.fsum equals the oracle, which uses the telescoped stresses;
  * the exact sum: the oracle's running sum stays within the classical bound
    n u sum |terms| of the correctly rounded sum;
  * layers below an element's bottom are never read; absent terms are zeros.
"""
import math
import os

import numpy as np
import pytest

import oracle
import sesynth

U_RND = 2.0 ** -53
GOLD = os.path.join(os.path.dirname(__file__), "golden", "forcing_column.txt")


def _golden():
    vals = {}
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        k, v = (t.strip() for t in line.split("="))
        if "|" in v:
            vals[k] = np.array([[float(x) for x in part.split()] for part in v.split("|")])
        else:
            nums = [float(x) for x in v.split()]
            vals[k] = np.array(nums) if len(nums) > 1 else nums[0]
    return vals


def test_hand_worked_column():
    g = _golden()
    K = int(g["K"])
    R = oracle.forcing(K=K, nlev=[int(g["nlev"])], RA=g["RA"][None], RP=g["RP"][None],
                       RhV=g["RhV"][None], tau_s=g["tau_s"][None], u=g["u"][None], Cd=g["Cd"])
    assert np.allclose(R[0], g["R"], rtol=0, atol=1e-14)


def _brute_layered(d, Av_rng):
    """eq. (eq4_4) term by term: per layer RA + RP + RhV + RvV, with RvV_k the stress on
    top of layer k minus the stress below it; the sum is exact (fsum)."""
    ne, K = d["nlev"].size, d["K"]
    out = np.empty((ne, 2))
    for e in range(ne):
        n = int(d["nlev"][e])
        ub = d["u"][e, n - 1]
        bottom = d["Cd"] * math.hypot(ub[0], ub[1]) * ub
        stress = [d["tau_s"][e]]
        for k in range(1, n):        # interface between layer k-1 (above) and k
            dz = 0.5 * (d["h"][e, k - 1] + d["h"][e, k])
            stress.append(Av_rng[e, k] * (d["u"][e, k - 1] - d["u"][e, k]) / dz)
        stress.append(bottom)
        for c in range(2):
            terms = []
            for k in range(n):
                rvv = stress[k][c] - stress[k + 1][c]
                terms += [d["RA"][e, k, c], d["RP"][e, k, c], d["RhV"][e, k, c], rvv]
            out[e, c] = math.fsum(terms)
    return out


@pytest.mark.parametrize("K", [1, 5, 40])
def test_per_layer_form_with_vertical_viscosity(K):
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=2, nsub=4)
    d = sesynth.column_forcing(case, K=K, seed=3)
    ne = d["nlev"].size
    r = sesynth.rng(77)
    d["h"] = 10.0 + 90.0 * r.random((ne, K))
    Av = 1e-4 + 1e-2 * r.random((ne, K))
    ref = _brute_layered(d, Av)
    R = oracle.forcing(K=K, nlev=d["nlev"], RA=d["RA"], RP=d["RP"], RhV=d["RhV"],
                       tau_s=d["tau_s"], u=d["u"], Cd=d["Cd"])
    # the interior stresses cancel only to rounding in the brute form
    scale = (np.abs(d["RA"]) + np.abs(d["RP"]) + np.abs(d["RhV"])).sum(axis=1) + 1e-4
    assert np.all(np.abs(R - ref) <= 1e-12 * scale)
    # the check sees the drag: twice the drag, or the drag on the layer above the
    # bottom, lands far outside that bound
    twice = oracle.forcing(K=K, nlev=d["nlev"], RA=d["RA"], RP=d["RP"], RhV=d["RhV"],
                           tau_s=d["tau_s"], u=d["u"], Cd=2 * d["Cd"])
    assert np.abs(twice - ref).max() > 1e3 * 1e-12 * scale.max()
    if K > 1:
        up = d["u"].copy()
        rows = np.nonzero(d["nlev"] > 1)[0]
        up[rows, d["nlev"][rows] - 1] = d["u"][rows, d["nlev"][rows] - 2]
        above = oracle.forcing(K=K, nlev=d["nlev"], RA=d["RA"], RP=d["RP"], RhV=d["RhV"],
                               tau_s=d["tau_s"], u=up, Cd=d["Cd"])
        assert np.abs(above - ref).max() > 1e3 * 1e-12 * scale.max()


def test_running_sum_within_the_classical_bound():
    case = sesynth.random_case(sesynth.tiny_mesh("sphere86"), seed=4, nsub=4)
    K = 40
    d = sesynth.column_forcing(case, K=K, seed=5)
    R = oracle.forcing(K=K, nlev=d["nlev"], RA=d["RA"], RP=d["RP"], RhV=d["RhV"],
                       tau_s=d["tau_s"], u=d["u"], Cd=d["Cd"])
    for e in range(d["nlev"].size):
        n = int(d["nlev"][e])
        ub = d["u"][e, n - 1]
        sp = math.hypot(ub[0], ub[1])
        for c in range(2):
            terms = [d["RA"][e, k, c] for k in range(n)] + [d["RP"][e, k, c] for k in range(n)] + \
                    [d["RhV"][e, k, c] for k in range(n)] + [d["tau_s"][e, c], -d["Cd"] * sp * ub[c]]
            exact = math.fsum(terms)
            bound = (len(terms) + 4) * U_RND * sum(abs(t) for t in terms)
            assert abs(R[e, c] - exact) <= bound


def test_padding_below_the_bottom_is_never_read():
    case = sesynth.random_case(sesynth.tiny_mesh("chan54"), seed=6, nsub=4)
    K = 12
    d = sesynth.column_forcing(case, K=K, seed=1)
    assert d["nlev"].min() < K
    pad = np.arange(K)[None, :] >= d["nlev"][:, None]
    args = {}
    for k in ("RA", "RP", "RhV", "u"):
        a = d[k].copy()
        a[pad] = np.nan
        args[k] = a
    R_nan = oracle.forcing(K=K, nlev=d["nlev"], tau_s=d["tau_s"], Cd=d["Cd"], **args)
    R = oracle.forcing(K=K, nlev=d["nlev"], RA=d["RA"], RP=d["RP"], RhV=d["RhV"],
                       tau_s=d["tau_s"], u=d["u"], Cd=d["Cd"])
    assert np.array_equal(R_nan, R)


def test_absent_terms_are_zero_and_single_layer_columns():
    r = sesynth.rng(9)
    ne, K = 17, 3
    RA = r.standard_normal((ne, K, 2))
    u = r.standard_normal((ne, K, 2))
    z = np.zeros((ne, K, 2))
    a = oracle.forcing(K=K, RA=RA, u=u, Cd=0.003)
    b = oracle.forcing(K=K, RA=RA, RP=z, RhV=z, tau_s=np.zeros((ne, 2)), u=u, Cd=0.003)
    assert np.array_equal(a, b)
    one = oracle.forcing(K=K, nlev=np.ones(ne, np.int32), RA=RA, u=u, Cd=0.003)
    sp = np.hypot(u[:, 0, 0], u[:, 0, 1])
    assert np.allclose(one, RA[:, 0] - 0.003 * sp[:, None] * u[:, 0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("bad", [0, 4, -1])
def test_out_of_range_layer_counts_are_rejected(bad):
    ne, K = 5, 3
    nlev = np.full(ne, 2, np.int32)
    nlev[3] = bad
    with pytest.raises(RuntimeError):
        oracle.forcing(K=K, nlev=nlev, RA=np.zeros((ne, K, 2)))
