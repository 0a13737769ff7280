"""GPU parity of the AB3-AM4 (SESM) subcycle, eqs. (eq4_7)-(eq4_8), against the
FP64 oracle through the C ABI.

FP64 bar: 1e-12 relative (same IEEE operations in the same order as the
oracle).  FP32 bar: e_max(eta) <= 1e-5 after about 1000 substeps, relative to
max |eta_oracle - eta_ref|.
"""
import numpy as np
import pytest

import oracle
import sesynth
from oracle import analytic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COEF = analytic.sesm_params(0.14)


def _params(case, precision="f64", **kw):
    from paper_2311_08241_amd import Params
    return Params(g=case["g"], theta=case["theta"], precision=precision,
                  linear_h=case["linear_h"], eta_ref=case["eta_ref"] if precision == "f32" else 0.0,
                  scheme="sesm", sesm=COEF, **kw)


def _run_gpu(case, mesh, params, nsteps, plain=True, W=None, plan=None):
    from paper_2311_08241_amd import device_inputs
    if plan is not None:
        mesh.set_plan(*plan)
    d = device_inputs(mesh, case, params)
    Wd = None if W is None else torch.tensor(mesh.v_in(W), dtype=params.dtype, device="cuda:0")
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    vols = []
    ws = mesh.workspace(params, case["nsub"])
    for _ in range(nsteps):
        vol = torch.empty(case["nsub"] + 1, dtype=torch.float64, device="cuda:0")
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], W=Wd, nsub=case["nsub"],
                      dt=case["tau"], params=params, Uavg=Uavg, volume=vol, workspace=ws,
                      plain=plain)
        vols.append(vol)
    torch.cuda.synchronize()
    assert mesh.check_faults() == 0
    eta = d["eta"].cpu().numpy().astype(np.float64)
    if params.precision == "f32":
        eta = eta + params.eta_ref
    vol = torch.cat([vols[0]] + [v[1:] for v in vols[1:]]).cpu().numpy()
    return (mesh.v_out(eta), mesh.e_out(d["U"].cpu().numpy().astype(np.float64)),
            mesh.e_out(Uavg.cpu().numpy()), vol)


def _run_oracle(case, nsteps, W=None):
    m = oracle.Mesh(case, reordered=True)
    eta, U = m.v_in(case["eta0"]), m.e_in(case["U0"])
    H0, f, R = m.v_in(case["H0"]), m.e_in(case["f"]), m.e_in(case["R"])
    Wi = None if W is None else m.v_in(W)
    b, d, g, z = COEF
    vols = []
    for _ in range(nsteps):
        eta, U, Uavg, vol = m.subcycle_sesm(eta, U, H0=H0, f=f, R=R, W=Wi, g=case["g"], beta=b,
                                            delta=d, gamma=g, zeta=z, nsub=case["nsub"],
                                            tau=case["tau"], linear_h=case["linear_h"])
        vols.append(vol if not vols else vol[1:])
    return m.v_out(eta), m.e_out(U), m.e_out(Uavg), np.concatenate(vols)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {}


def _case(name):
    if name not in CASES:
        if name in ("jitter76", "chan54", "sphere86", "torus43"):
            c = sesynth.random_case(sesynth.tiny_mesh(name), seed=3, nsub=18)
            if name == "sphere86":
                c["tau"] = 18 * 20.0
        elif name == "fan100":   # one vertex shared by 100 triangles
            c = sesynth.random_case(sesynth.tiny_mesh("fan100"), seed=3, nsub=18, tau=2.7)
        elif name == "C1":
            c = sesynth.basin_c1()
        elif name == "C2s":
            c = sesynth.channel_c2(nx=256, ny=128, nsteps=4)
        elif name == "C3s":
            c = sesynth.latlon_c3(nlon=256, nlat=192, nsteps=2)
            c["tau"] = c["nsub"] * 90.0
        else:
            raise KeyError(name)
        CASES[name] = c
    return CASES[name]


def test_library_coefficients_match_the_paper_settings():
    from paper_2311_08241_amd.api import sesm_coefficients
    assert np.allclose(sesm_coefficients(0.14), COEF, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["jitter76", "chan54", "sphere86", "torus43", "fan100", "C1", "C2s",
                                  "C3s"])
def test_sesm_fp64_plain_matches_oracle(name):
    from paper_2311_08241_amd import Mesh
    case = _case(name)
    nsteps = 2
    W = 1e-5 * sesynth.rng(5).standard_normal(case["x"].size) if name == "jitter76" else None
    mesh = Mesh.from_dict(case, device=0)
    eta, U, Uavg, vol = _run_gpu(case, mesh, _params(case), nsteps, W=W)
    eta_r, U_r, Uavg_r, vol_r = _run_oracle(case, nsteps, W=W)
    assert _rel(eta, eta_r) <= 1e-12
    assert _rel(U, U_r) <= 1e-12
    assert _rel(Uavg, Uavg_r) <= 1e-12
    assert np.abs(vol - vol_r).max() <= 1e-12 * np.abs(vol_r).max()


def test_sesm_fp32_plain_budget_c2():
    from paper_2311_08241_amd import Mesh
    case = sesynth.channel_c2(nx=256, ny=128, nsteps=17)
    mesh = Mesh.from_dict(case, device=0)
    eta, U, Uavg, _ = _run_gpu(case, mesh, _params(case, "f32"), 17)     # 1020 substeps
    eta_r, U_r, Uavg_r, _ = _run_oracle(case, 17)
    e_max = np.abs(eta - eta_r).max() / np.abs(eta_r - case["eta_ref"]).max()
    assert e_max <= 1e-5, e_max
    assert _rel(Uavg, Uavg_r) <= 1e-4


def test_sesm_volume_conserved_on_gpu():
    from paper_2311_08241_amd import Mesh
    case = _case("C1")
    mesh = Mesh.from_dict(case, device=0)
    _, _, _, vol = _run_gpu(case, mesh, _params(case), 3)
    atot = mesh.geometry()[0].sum()
    assert np.abs(vol - vol[0]).max() <= 1e-13 * atot * np.abs(case["eta0"]).max()


def test_sesm_cfl_check_uses_the_sesm_limit():
    from paper_2311_08241_amd import Mesh, device_inputs
    import paper_2311_08241_amd._lib as L
    case = _case("C1")
    mesh = Mesh.from_dict(case, device=0)
    lim = analytic.sesm_stability_limit(*COEF)
    hmax = float(np.max(case["H0"] + np.abs(case["eta0"])))
    for frac, ok in ((0.97, True), (1.03, False)):
        dts = frac * lim / np.sqrt(case["g"] * hmax * mesh.mu_max)
        p = _params(case, check_cfl=True, h_max=hmax)
        d = device_inputs(mesh, case, p)
        ws = mesh.workspace(p, 4)
        try:
            mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=4, dt=4 * dts,
                          params=p, workspace=ws, plain=True)
            torch.cuda.synchronize()
            raised = False
        except L.SeError as e:
            assert e.status == L.SE_ERR_CFL
            raised = True
        assert raised == (not ok)


PLANS = [(64, 1, 256), (64, 3, 256), (128, 4, 256), (256, 2, 512), (96, 8, 256)]


def _plans_ok(mesh, prec):
    out = []
    for pl in PLANS:
        if mesh.plan_stats(*pl)["ok_sesm_" + prec]:
            out.append(pl)
    assert out, "no plan fits"
    return out


@pytest.mark.parametrize("name", ["jitter76", "chan54", "sphere86", "torus43", "fan100", "C1", "C2s",
                                  "C3s"])
def test_sesm_fp64_tile_matches_oracle(name):
    from paper_2311_08241_amd import Mesh
    case = _case(name)
    nsteps = 2
    W = 1e-5 * sesynth.rng(5).standard_normal(case["x"].size) if name == "jitter76" else None
    mesh = Mesh.from_dict(case, device=0)
    eta_r, U_r, Uavg_r, vol_r = _run_oracle(case, nsteps, W=W)
    for pl in _plans_ok(mesh, "f64"):
        eta, U, Uavg, vol = _run_gpu(case, mesh, _params(case), nsteps, plain=False, W=W, plan=pl)
        assert _rel(eta, eta_r) <= 1e-12, pl
        assert _rel(U, U_r) <= 1e-12, pl
        assert _rel(Uavg, Uavg_r) <= 1e-12, pl
        assert np.abs(vol - vol_r).max() <= 1e-12 * np.abs(vol_r).max(), pl


def test_sesm_fp32_tile_identical_to_plain_and_across_plans():
    from paper_2311_08241_amd import Mesh
    case = _case("C2s")
    mesh = Mesh.from_dict(case, device=0)
    p = _params(case, "f32")
    ref = _run_gpu(case, mesh, p, 2, plain=True)
    for pl in _plans_ok(mesh, "f32"):
        out = _run_gpu(case, mesh, p, 2, plain=False, plan=pl)
        for a, b in zip(out[:3], ref[:3]):
            assert np.array_equal(a, b), pl


@pytest.mark.parametrize("nsub", [1, 5, 7])
def test_sesm_tile_partial_chunks(nsub):
    """nsub below, between and not divisible by the substeps per launch."""
    from paper_2311_08241_amd import Mesh
    case = dict(_case("jitter76"))
    case["tau"] = case["tau"] / case["nsub"] * nsub
    case["nsub"] = nsub
    mesh = Mesh.from_dict(case, device=0)
    eta_r, U_r, Uavg_r, _ = _run_oracle(case, 1)
    for pl in _plans_ok(mesh, "f64"):
        eta, U, Uavg, _ = _run_gpu(case, mesh, _params(case), 1, plain=False, plan=pl)
        assert _rel(eta, eta_r) <= 1e-12 and _rel(U, U_r) <= 1e-12, (pl, nsub)
        assert _rel(Uavg, Uavg_r) <= 1e-12, (pl, nsub)
