"""GPU parity of the barotropic viscous regularization, eq. (eq:viscosity_BT), and
of the plain subcycle that carries it (its initial value subtracted from R),
against the FP64 oracle through the C ABI.

FP64 bar: 1e-12 relative (same operations in the same order as the oracle).
FP32: the operator within 1e-5 of max |V|; the subcycle within the FP32 budget
e_max(eta) <= 1e-5 after about 1000 substeps.
"""
import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KINDS = ["jitter76", "chan54", "sphere86", "torus43"]


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _t(a, dt=torch.float64):
    return torch.tensor(a, dtype=dt, device="cuda:0")


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("A0,Cv,linear_h", [(300.0, 0.0, False), (50.0, 0.2, False),
                                            (0.0, 0.5, True)])
def test_operator_matches_oracle(kind, A0, Cv, linear_h):
    from paper_2311_08241_amd import Mesh
    c = sesynth.random_case(sesynth.tiny_mesh(kind), seed=3, nsub=16)
    mesh = Mesh.from_dict(c, device=0)
    om = oracle.Mesh(c, reordered=True)
    H0, eta, U = om.v_in(c["H0"]), om.v_in(c["eta0"]), om.e_in(c["U0"])
    ref = om.visc(eta, U, H0=H0, A0=A0, Cv=Cv, linear_h=linear_h)
    V = mesh.visc(_t(eta), _t(U), H0=_t(H0), A0=A0, Cv=Cv, linear_h=linear_h)
    torch.cuda.synchronize()
    assert _rel(V.cpu().numpy(), ref) <= 1e-12
    # FP32 form: eta as the deviation from eta_ref
    ref_eta = float(np.mean(eta))
    f = torch.float32
    V32 = mesh.visc(_t(eta - ref_eta, f), _t(U, f), H0=_t(H0, f), A0=A0, Cv=Cv,
                    precision="f32", linear_h=linear_h, eta_ref=ref_eta)
    torch.cuda.synchronize()
    assert _rel(V32.cpu().numpy().astype(np.float64), ref) <= 1e-5


def _params(case, precision, visc):
    from paper_2311_08241_amd import Params
    return Params(g=case["g"], theta=case["theta"], precision=precision,
                  linear_h=case["linear_h"], eta_ref=case["eta_ref"] if precision == "f32" else 0.0,
                  visc=visc)


def _run_gpu(case, mesh, p, nsteps, W=None):
    from paper_2311_08241_amd import device_inputs
    d = device_inputs(mesh, case, p)
    Wd = None if W is None else torch.tensor(mesh.v_in(W), dtype=p.dtype, device="cuda:0")
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    ws = mesh.workspace(p, case["nsub"])
    vols = []
    for _ in range(nsteps):
        vol = torch.empty(case["nsub"] + 1, dtype=torch.float64, device="cuda:0")
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], W=Wd, nsub=case["nsub"],
                      dt=case["tau"], params=p, Uavg=Uavg, volume=vol, workspace=ws, plain=True)
        vols.append(vol)
    torch.cuda.synchronize()
    assert mesh.check_faults() == 0
    eta = d["eta"].cpu().numpy().astype(np.float64)
    if p.precision == "f32":
        eta = eta + p.eta_ref
    vol = torch.cat([vols[0]] + [v[1:] for v in vols[1:]]).cpu().numpy()
    return (mesh.v_out(eta), mesh.e_out(d["U"].cpu().numpy().astype(np.float64)),
            mesh.e_out(Uavg.cpu().numpy()), vol)


def _run_oracle(case, nsteps, visc, W=None):
    m = oracle.Mesh(case, reordered=True)
    eta, U = m.v_in(case["eta0"]), m.e_in(case["U0"])
    H0, f, R = m.v_in(case["H0"]), m.e_in(case["f"]), m.e_in(case["R"])
    Wi = None if W is None else m.v_in(W)
    vols = []
    for _ in range(nsteps):
        eta, U, Uavg, vol = m.subcycle(eta, U, H0=H0, f=f, R=R, W=Wi, g=case["g"],
                                       theta=case["theta"], nsub=case["nsub"], tau=case["tau"],
                                       linear_h=case["linear_h"], visc=visc)
        vols.append(vol if not vols else vol[1:])
    return m.v_out(eta), m.e_out(U), m.e_out(Uavg), np.concatenate(vols)


def _case(name):
    if name == "fan100":   # sliver triangles around a vertex shared by 100 of them
        c = sesynth.random_case(sesynth.tiny_mesh("fan100"), seed=7, nsub=16, tau=2.4)
        m = oracle.Mesh(c, reordered=False)
        nb, l, lod = m.visc_geometry()
        # a tenth of the explicit limit dt_s A0 max_e sum_j (l/d)_j / A_e ~ 1
        return c, (0.1 / (c["tau"] / c["nsub"] * np.max(lod.sum(1) / m.Ae)), 0.0)
    if name in KINDS:
        c = sesynth.random_case(sesynth.tiny_mesh(name), seed=7, nsub=16)
        Ae = oracle.Mesh(c, reordered=False).Ae.mean()
        return c, (0.02 * Ae * c["nsub"] / c["tau"], 0.5)
    if name == "C1":
        return sesynth.basin_c1(), (2.0e4, 0.2)
    if name == "C2s":
        return sesynth.channel_c2(nx=256, ny=128, nsteps=4), (200.0, 0.1)
    if name == "C3s":
        c = sesynth.latlon_c3(nlon=256, nlat=192, nsteps=2)
        return c, (2.0e3, 0.1)
    raise KeyError(name)


@pytest.mark.parametrize("name", KINDS + ["fan100", "C1", "C2s", "C3s"])
def test_viscous_subcycle_fp64_matches_oracle(name):
    from paper_2311_08241_amd import Mesh
    case, visc = _case(name)
    W = 1e-5 * sesynth.rng(5).standard_normal(case["x"].size) if name == "jitter76" else None
    mesh = Mesh.from_dict(case, device=0)
    out = _run_gpu(case, mesh, _params(case, "f64", visc), 2, W=W)
    ref = _run_oracle(case, 2, visc, W=W)
    for a, b in zip(out[:3], ref[:3]):
        assert _rel(a, b) <= 1e-12
    assert np.abs(out[3] - ref[3]).max() <= 1e-12 * np.abs(ref[3]).max()


def test_viscous_subcycle_fp32_budget_c2():
    from paper_2311_08241_amd import Mesh
    case = sesynth.channel_c2(nx=256, ny=128, nsteps=17)
    visc = (200.0, 0.1)
    mesh = Mesh.from_dict(case, device=0)
    eta, U, Uavg, _ = _run_gpu(case, mesh, _params(case, "f32", visc), 17)   # 1020 substeps
    eta_r, U_r, Uavg_r, _ = _run_oracle(case, 17, visc)
    e_max = np.abs(eta - eta_r).max() / np.abs(eta_r - case["eta_ref"]).max()
    assert e_max <= 1e-5, e_max
    assert _rel(Uavg, Uavg_r) <= 1e-4


def test_viscous_lake_at_rest_exact_on_gpu():
    from paper_2311_08241_amd import Mesh
    c = sesynth.random_case(sesynth.tiny_mesh("sphere86"), seed=3, nsub=16)
    c["eta0"] = np.full_like(c["eta0"], 0.5)
    c["U0"] = np.zeros_like(c["U0"])
    c["R"] = np.zeros_like(c["R"])
    mesh = Mesh.from_dict(c, device=0)
    eta, U, Uavg, _ = _run_gpu(c, mesh, _params(c, "f64", (1.0e6, 0.5)), 1)
    assert np.all(eta == 0.5) and np.all(U == 0.0) and np.all(Uavg == 0.0)


def test_viscous_term_is_refused_where_not_implemented():
    import paper_2311_08241_amd._lib as L
    from paper_2311_08241_amd import Mesh, Params, device_inputs
    c = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=3, nsub=8)
    mesh = Mesh.from_dict(c, device=0)
    p = _params(c, "f64", (100.0, 0.1))
    d = device_inputs(mesh, c, p)
    ws = mesh.workspace(p, c["nsub"])
    # the tile form needs two rings per substep
    mesh.set_plan(64, 1, 256)
    with pytest.raises(L.SeError) as ei:
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=c["nsub"],
                      dt=c["tau"], params=p, workspace=ws, plain=False)
    assert ei.value.status == L.SE_ERR_ARG
    ps = Params(g=c["g"], theta=c["theta"], scheme="sesm", visc=(100.0, 0.1))
    for plain in (True, False):
        with pytest.raises(L.SeError) as ei:
            mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=c["nsub"],
                          dt=c["tau"], params=ps, workspace=mesh.workspace(ps, c["nsub"]),
                          plain=plain)
        assert ei.value.status == L.SE_ERR_UNSUPPORTED
    bad = _params(c, "f64", (-1.0, 0.0))
    with pytest.raises(L.SeError) as ei:
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=c["nsub"],
                      dt=c["tau"], params=bad, workspace=ws, plain=True)
    assert ei.value.status == L.SE_ERR_ARG
    torch.cuda.synchronize()


# tile plans with at least two rings: (64, 3) and (256, 2) run one viscous substep per
# launch, (128, 4) two, (96, 8) four
VPLANS = [(64, 3, 256), (128, 4, 256), (256, 2, 512), (96, 8, 256)]


def _run_tile(case, mesh, p, nsteps, plan, W=None):
    mesh.set_plan(*plan)
    from paper_2311_08241_amd import device_inputs
    d = device_inputs(mesh, case, p)
    Wd = None if W is None else torch.tensor(mesh.v_in(W), dtype=p.dtype, device="cuda:0")
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    ws = mesh.workspace(p, case["nsub"])
    vols = []
    for _ in range(nsteps):
        vol = torch.empty(case["nsub"] + 1, dtype=torch.float64, device="cuda:0")
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], W=Wd, nsub=case["nsub"],
                      dt=case["tau"], params=p, Uavg=Uavg, volume=vol, workspace=ws, plain=False)
        vols.append(vol)
    torch.cuda.synchronize()
    assert mesh.check_faults() == 0
    eta = d["eta"].cpu().numpy().astype(np.float64)
    if p.precision == "f32":
        eta = eta + p.eta_ref
    vol = torch.cat([vols[0]] + [v[1:] for v in vols[1:]]).cpu().numpy()
    return (mesh.v_out(eta), mesh.e_out(d["U"].cpu().numpy().astype(np.float64)),
            mesh.e_out(Uavg.cpu().numpy()), vol)


@pytest.mark.parametrize("name", KINDS + ["fan100", "C1", "C2s", "C3s"])
def test_viscous_tile_fp64_matches_oracle(name):
    from paper_2311_08241_amd import Mesh
    case, visc = _case(name)
    W = 1e-5 * sesynth.rng(5).standard_normal(case["x"].size) if name == "jitter76" else None
    mesh = Mesh.from_dict(case, device=0)
    ref = _run_oracle(case, 2, visc, W=W)
    for pl in VPLANS:
        if not mesh.plan_stats(*pl)["ok_f64"]:
            continue
        out = _run_tile(case, mesh, _params(case, "f64", visc), 2, pl, W=W)
        for a, b in zip(out[:3], ref[:3]):
            assert _rel(a, b) <= 1e-12, pl
        assert np.abs(out[3] - ref[3]).max() <= 1e-12 * np.abs(ref[3]).max(), pl


def test_viscous_tile_fp32_identical_to_plain():
    from paper_2311_08241_amd import Mesh
    case, visc = _case("C2s")
    mesh = Mesh.from_dict(case, device=0)
    p = _params(case, "f32", visc)
    ref = _run_gpu(case, mesh, p, 2)
    # and the FP32 register tiers of the viscous form: three triangles per thread with
    # 1024- and 512-thread workgroups
    for pl in VPLANS + [(512, 6, 1024), (256, 4, 512)]:
        if not mesh.plan_stats(*pl)["ok_f32"]:
            continue
        out = _run_tile(case, mesh, p, 2, pl)
        for a, b in zip(out[:3], ref[:3]):
            assert np.array_equal(a, b), pl


@pytest.mark.parametrize("nsub", [1, 3, 5])
def test_viscous_tile_partial_chunks(nsub):
    """nsub below, at and not divisible by the substeps per launch."""
    from paper_2311_08241_amd import Mesh
    case, visc = _case("jitter76")
    case = dict(case)
    case["tau"] = case["tau"] / case["nsub"] * nsub
    case["nsub"] = nsub
    mesh = Mesh.from_dict(case, device=0)
    ref = _run_oracle(case, 1, visc)
    for pl in VPLANS:
        out = _run_tile(case, mesh, _params(case, "f64", visc), 1, pl)
        for a, b in zip(out[:3], ref[:3]):
            assert _rel(a, b) <= 1e-12, (pl, nsub)
