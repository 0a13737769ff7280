"""GPU parity of the vertically integrated baroclinic forcing, eq. (eq4_4), against
the FP64 oracle through the C ABI.

Bar: per triangle and component, |R_gpu - R_oracle| <= 2 (3 n + 6) u S, with n the
triangle's layer count, u = 2^-53 and S the sum of the magnitudes of every term
(the layer tendencies, the surface stress and the drag): both sides sum the same
terms in different orders (the GPU adds eight strided partial sums by a
butterfly), and each order is within (3 n + 6) u S of the exact sum.  The FP32
output is the float rounding of the GPU's FP64 sum, bit for bit.
"""
import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U_RND = 2.0 ** -53


def _bound(d):
    K = d["K"]
    n = d["nlev"]
    act = (np.arange(K)[None, :] < n[:, None])[:, :, None]
    S = sum(np.where(act, np.abs(d[k]), 0.0).sum(axis=1) for k in ("RA", "RP", "RhV"))
    ub = d["u"][np.arange(n.size), n - 1]
    sp = np.hypot(ub[:, 0], ub[:, 1])
    S = S + np.abs(d["tau_s"]) + d["Cd"] * sp[:, None] * np.abs(ub)
    return 2.0 * (3 * n[:, None] + 6) * U_RND * S


def _dev(a, dtype=torch.float64):
    return None if a is None else torch.tensor(a, dtype=dtype, device="cuda:0")


def _gpu(mesh, d, precision="f64", drop=()):
    args = {k: (None if k in drop else _dev(d[k])) for k in ("RA", "RP", "RhV", "tau_s", "u")}
    nlev = None if "nlev" in drop else _dev(d["nlev"], torch.int32)
    R = mesh.forcing(K=d["K"], nlev=nlev, Cd=d["Cd"], precision=precision, **args)
    torch.cuda.synchronize()
    return R.cpu().numpy()


def _orc(d, drop=()):
    args = {k: (None if k in drop else d[k]) for k in ("RA", "RP", "RhV", "tau_s", "u")}
    return oracle.forcing(K=d["K"], nlev=None if "nlev" in drop else d["nlev"], Cd=d["Cd"],
                          **args)


@pytest.mark.parametrize("kind,K", [("jitter76", 1), ("chan54", 5), ("sphere86", 12),
                                    ("torus43", 40), ("jitter76", 70)])
def test_forcing_matches_oracle(kind, K):
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh(kind), seed=2, nsub=4)
    d = sesynth.column_forcing(case, K=K, seed=K)
    mesh = Mesh.from_dict(case, device=0)
    R = _gpu(mesh, d)
    ref = _orc(d)
    assert np.all(np.abs(R - ref) <= _bound(d))
    R32 = _gpu(mesh, d, "f32")
    assert R32.dtype == np.float32 and np.array_equal(R32, R.astype(np.float32))
    assert mesh.check_faults() == 0


def test_forcing_padding_not_read_and_absent_terms():
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh("chan54"), seed=3, nsub=4)
    K = 16
    d = sesynth.column_forcing(case, K=K, seed=8)
    assert d["nlev"].min() < K
    mesh = Mesh.from_dict(case, device=0)
    ref = _gpu(mesh, d)
    pad = np.arange(K)[None, :] >= d["nlev"][:, None]
    dn = dict(d)
    for k in ("RA", "RP", "RhV", "u"):
        dn[k] = d[k].copy()
        dn[k][pad] = np.nan
    assert np.array_equal(_gpu(mesh, dn), ref)
    for drop in (("RP",), ("RA", "RhV"), ("tau_s",)):
        R = _gpu(mesh, d, drop=drop)
        assert np.all(np.abs(R - _orc(d, drop=drop)) <= _bound(d))
    # no layer counts: every column has K layers
    full = dict(d, nlev=np.full(d["nlev"].size, K, np.int32))
    R = _gpu(mesh, d, drop=("nlev",))
    assert np.all(np.abs(R - _orc(full)) <= _bound(full))
    # no drag: u may be absent
    d0 = dict(d, Cd=0.0)
    R = _gpu(mesh, d0, drop=("u",))
    assert np.all(np.abs(R - _orc(d0, drop=("u",))) <= _bound(d0))
    assert mesh.check_faults() == 0


def test_forcing_bad_layer_count_faults_that_triangle_only():
    import paper_2311_08241_amd._lib as L
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=4, nsub=4)
    K = 8
    d = sesynth.column_forcing(case, K=K, seed=2)
    mesh = Mesh.from_dict(case, device=0)
    ref = _gpu(mesh, d)
    bad = dict(d, nlev=d["nlev"].copy())
    bad["nlev"][[3, 10]] = [0, K + 1]
    R = _gpu(mesh, bad)
    assert mesh.check_faults() == L.SE_FAULT_LAYERS
    assert np.all(np.isnan(R[[3, 10]]))
    keep = np.setdiff1d(np.arange(R.shape[0]), [3, 10])
    assert np.array_equal(R[keep], ref[keep])


def test_forcing_rejects_bad_arguments():
    import paper_2311_08241_amd._lib as L
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=4, nsub=4)
    d = sesynth.column_forcing(case, K=4, seed=2)
    mesh = Mesh.from_dict(case, device=0)
    with pytest.raises(L.SeError):
        _gpu(mesh, dict(d, Cd=-1.0))
    with pytest.raises(L.SeError):
        _gpu(mesh, d, drop=("u",))          # Cd > 0 needs u
    with pytest.raises(ValueError):
        mesh.forcing(K=5, RA=_dev(d["RA"]))  # shape does not match K
