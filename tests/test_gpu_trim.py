"""GPU parity of the consumer of the averaged transport (trim of layer
transports, eq. (eq4_13); z* thicknesses and diasurface velocity, Sec. 2.4)
against the FP64 oracle through the C ABI, bar 1e-12 relative (the sums over
layers and the vertical recursion differ from the definition only in rounding
order).
"""
import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(case, K, seed, with_w):
    om = oracle.Mesh(case, reordered=True)
    H0 = om.v_in(case["H0"])
    eta0 = om.v_in(case["eta0"])
    W = 1e-5 * sesynth.rng(31).standard_normal(case["x"].size) if with_w else None
    Wi = None if W is None else om.v_in(W)
    eta1, _, Uavg, _ = om.subcycle(eta0, om.e_in(case["U0"]), H0=H0, f=om.e_in(case["f"]),
                                   R=om.e_in(case["R"]), W=Wi, g=case["g"], theta=case["theta"],
                                   nsub=case["nsub"], tau=case["tau"], volume=False)
    lay = sesynth.layers(case, K=K, seed=seed)
    Ustar = lay["Ustar"][om.eperm]
    h0 = H0[:, None] * lay["frac"][None, :]
    hn = h0 * ((H0 + eta0) / H0)[:, None]
    return om, dict(H0=H0, eta_new=eta1, Uavg=Uavg, Ustar=np.ascontiguousarray(Ustar), hn=hn,
                    h0=h0, W=Wi, tau=case["tau"])


def _gpu(mesh, inp, inplace=False):
    t = {k: (None if v is None else
             torch.tensor(v, dtype=torch.float64, device="cuda:0") if isinstance(v, np.ndarray)
             else v) for k, v in inp.items()}
    U = t["Ustar"] if inplace else None
    U, hnew, w = mesh.trim_zstar(H0=t["H0"], eta_new=t["eta_new"], Uavg=t["Uavg"],
                                 Ustar=t["Ustar"], hn=t["hn"], h0=t["h0"], W=t["W"],
                                 tau=t["tau"], U=U)
    torch.cuda.synchronize()
    return U.cpu().numpy(), hnew.cpu().numpy(), w.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86"])
@pytest.mark.parametrize("with_w", [False, True])
def test_trim_matches_oracle_small(kind, with_w):
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh(kind), seed=4, nsub=24)
    om, inp = _inputs(case, 12, 1, with_w)
    mesh = Mesh.from_dict(case, device=0)
    ref = om.trim_zstar(**inp)
    out = _gpu(mesh, inp)
    for a, b in zip(out, ref):
        assert _rel(a, b) <= 1e-12


@pytest.mark.parametrize("K", [1, 2, 9, 20, 27, 45, 55, 63, 64])
def test_trim_layer_count_limits(K):
    """One layer (the trim is then U = <<U>>), the largest column the kernels take, and
    every count of layers per lane (ceil(K / 8) = 1 .. 8, ragged last block)."""
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh("chan54"), seed=4, nsub=24)
    om, inp = _inputs(case, K, 3, True)
    mesh = Mesh.from_dict(case, device=0)
    ref = om.trim_zstar(**inp)
    out = _gpu(mesh, inp)
    for a, b in zip(out[:2], ref[:2]):
        assert _rel(a, b) <= 1e-12
    # w: with one layer only the surface value exists, the column closure, which is
    # rounding noise; measure against the size of the terms it sums
    wscale = max(np.abs(ref[2]).max(), np.abs(ref[1] - inp["hn"]).sum(1).max() / inp["tau"])
    assert np.abs(out[2] - ref[2]).max() <= 1e-12 * wscale
    if K == 1:
        assert _rel(out[0][:, 0], inp["Uavg"]) <= 1e-14


@pytest.mark.parametrize("K", [24, 40])
def test_trim_long_csr_row(K):
    """A vertex shared by 100 triangles: its CSR row spans more than one window of
    columns.  With 24 layers its row fits one tile of the one-launch form (128 local
    triangles); with 40 (64 per tile) it does not, and the three-launch form runs."""
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh("fan100"), seed=4, nsub=24, tau=4.0)
    om, inp = _inputs(case, K, 1, True)
    mesh = Mesh.from_dict(case, device=0)
    ref = om.trim_zstar(**inp)
    out = _gpu(mesh, inp)
    for a, b in zip(out, ref):
        assert _rel(a, b) <= 1e-12


def test_trim_c2_forty_layers_both_forms_and_closure():
    """The channel workload at 40 layers: out of place (the one-launch tile form) and in
    place (U = Ustar: the three-launch form) against the oracle, and against each other
    bit for bit (the same operations in the same order)."""
    from paper_2311_08241_amd import Mesh
    case = sesynth.channel_c2(nsteps=1)
    om, inp = _inputs(case, 40, 2, True)
    mesh = Mesh.from_dict(case, device=0)
    ref = om.trim_zstar(**inp)
    tiled = _gpu(mesh, inp)
    out = _gpu(mesh, inp, inplace=True)
    for a, b, c in zip(out, ref, tiled):
        assert _rel(a, b) <= 1e-12
        assert np.array_equal(a, c)
    # column closure at the surface (eq. (eq4_11)-(eq4_13))
    assert np.abs(out[2][:, 0]).max() <= 1e-12 * inp["H0"].max() / inp["tau"]


@pytest.mark.parametrize("K", [1, 8, 9, 17, 24, 25, 33, 40, 41, 49, 64])
def test_trim_tile_form_equals_three_launch_form_bitwise(K):
    """Every layer count class of the tile form (triangles per tile 256, 128, 96, 64) on
    a mesh of many tiles, bit for bit against the three-launch form (in place)."""
    from paper_2311_08241_amd import Mesh
    case = sesynth.channel_c2(nx=96, ny=40, nsteps=1)
    om, inp = _inputs(case, K, 5, True)
    mesh = Mesh.from_dict(case, device=0)
    tiled = _gpu(mesh, inp)
    out = _gpu(mesh, inp, inplace=True)
    for a, c in zip(out, tiled):
        assert np.array_equal(a, c)


def test_trim_rejects_bad_arguments():
    import paper_2311_08241_amd._lib as L
    from paper_2311_08241_amd import Mesh
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=4, nsub=24)
    om, inp = _inputs(case, 12, 1, False)
    mesh = Mesh.from_dict(case, device=0)
    inp["tau"] = 0.0
    with pytest.raises(L.SeError):
        _gpu(mesh, inp)
