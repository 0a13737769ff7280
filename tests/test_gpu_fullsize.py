"""Parity at the workloads' full sizes, in the launch configurations the
benchmark selects (tile plans of the autotuner's shortlist).

  lat-lon 2048x1536, 30% land (2.2M vertices): FP64 one step equal to the
      oracle to 1e-12; FP32 identical across plans (the benchmark's timed plan
      464,4,512 and the ensemble's 352,4,512 among them), and within 1e-5 of the
      oracle after 1040 substeps
  channel 1024x512 (0.5M vertices): FP32 within 1e-5 after 1020 substeps
  adjoint basin 256x256: FP64 adjoint equal to the oracle's to 1e-12
  ensemble of 64 basins (10k-200k vertices, 20-120 substeps): every member of
      the batched run against the oracle after 10 steps, FP64 within 1e-12 and
      FP32 within 1e-5
  AB3-AM4 (SESM) scheme: lat-lon FP64 one step equal to the oracle to 1e-12;
      channel FP32 within 1e-5 of the oracle after 1020 substeps
  consumers at 40 layers on the lat-lon mesh: vertically integrated forcing within
      the summation bound of the oracle; trim/z* within 1e-12
"""
import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_CACHE = {}


def _c3():
    if "c3" not in _CACHE:
        from paper_2311_08241_amd import Mesh
        case = sesynth.latlon_c3()
        _CACHE["c3"] = (case, Mesh.from_dict(case, device=0), oracle.Mesh(case, reordered=True))
    return _CACHE["c3"]


def _gpu_steps(mesh, case, prec, plan, nsteps):
    from paper_2311_08241_amd import Params, device_inputs
    mesh.set_plan(*plan)
    p = Params(precision=prec, eta_ref=case["eta_ref"] if prec == "f32" else 0.0)
    d = device_inputs(mesh, case, p)
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    ws = mesh.workspace(p, case["nsub"])
    for _ in range(nsteps):
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"],
                      dt=case["tau"], params=p, Uavg=Uavg, workspace=ws)
    torch.cuda.synchronize()
    assert mesh.check_faults() == 0
    eta = d["eta"].double().cpu().numpy() + p.eta_ref
    return mesh.v_out(eta), mesh.e_out(Uavg.cpu().numpy())


def _oracle_steps(om, case, nsteps):
    H0, f, R = om.v_in(case["H0"]), om.e_in(case["f"]), om.e_in(case["R"])
    eta, U = om.v_in(case["eta0"]), om.e_in(case["U0"])
    for _ in range(nsteps):
        eta, U, Uavg, _ = om.subcycle(eta, U, H0=H0, f=f, R=R, g=case["g"], theta=case["theta"],
                                      nsub=case["nsub"], tau=case["tau"], volume=False,
                                      threads=0)
    return om.v_out(eta), om.e_out(Uavg)


# the benchmark's timed plan first (its errors are the ones asserted), then other
# tile shapes, the ensemble's shipped plan among them
FP32_PLANS = [(520, 4, 512), (768, 6, 512), (512, 8, 512), (768, 5, 512), (448, 4, 512),
              (464, 4, 512)]


def test_c3_fp64_one_step_equals_oracle():
    case, mesh, om = _c3()
    eta_r, ua_r = _oracle_steps(om, case, 1)
    for plan in ((384, 4, 512), (512, 3, 512)):
        eta, ua = _gpu_steps(mesh, case, "f64", plan, 1)
        assert np.abs(eta - eta_r).max() <= 1e-12 * np.abs(eta_r).max()
        assert np.abs(ua - ua_r).max() <= 1e-12 * np.abs(ua_r).max()


def test_c3_fp32_identical_across_plans_and_1040_substep_budget():
    case, mesh, om = _c3()
    nsteps = 13      # 13 x 80 = 1040 substeps
    outs = [_gpu_steps(mesh, case, "f32", p, nsteps) for p in FP32_PLANS]
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    eta_r, ua_r = _oracle_steps(om, case, nsteps)
    e_max = np.abs(outs[0][0] - eta_r).max() / np.abs(eta_r - case["eta_ref"]).max()
    u_max = np.abs(outs[0][1] - ua_r).max() / np.abs(ua_r).max()
    print(f"lat-lon FP32 after 1040 substeps: eta e_max {e_max:.2e}, <<U>> e_max {u_max:.2e}",
          flush=True)
    assert e_max <= 1e-5, e_max
    assert u_max <= 1e-5, u_max


def test_c2_fp32_1020_substep_budget():
    from paper_2311_08241_amd import Mesh
    case = sesynth.channel_c2(nsteps=17)
    mesh = Mesh.from_dict(case, device=0)
    om = oracle.Mesh(case, reordered=True)
    eta, ua = _gpu_steps(mesh, case, "f32", (768, 6, 512), 17)
    eta_r, ua_r = _oracle_steps(om, case, 17)
    e_max = np.abs(eta - eta_r).max() / np.abs(eta_r - case["eta_ref"]).max()
    assert e_max <= 1e-5, e_max
    eta64, ua64 = _gpu_steps(mesh, case, "f64", (384, 4, 512), 1)
    eta_r1, ua_r1 = _oracle_steps(om, case, 1)
    assert np.abs(eta64 - eta_r1).max() <= 1e-12 * np.abs(eta_r1).max()


def test_c5_adjoint_full_size_equals_oracle():
    from paper_2311_08241_amd import Mesh, Params, device_inputs
    case = sesynth.adjoint_c5()
    mesh = Mesh.from_dict(case, device=0)
    om = oracle.Mesh(case, reordered=True)
    p = Params(precision="f64")
    d = device_inputs(mesh, case, p)
    eta, U = d["eta"].clone(), d["U"].clone()
    mesh.subcycle(eta, U, R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"], dt=case["tau"],
                  params=p)
    Av = torch.tensor(mesh.geometry()[0], dtype=torch.float64, device="cuda:0")
    tgt = torch.tensor(mesh.v_in(case["eta_target"]), dtype=torch.float64, device="cuda:0")
    lam = 2 * Av * (eta - tgt)
    lam_o = om.v_in(mesh.v_out(lam.cpu().numpy()))
    ref = om.adjoint(om.v_in(case["eta0"]), om.e_in(case["U0"]), lam_o, H0=om.v_in(case["H0"]),
                     f=om.e_in(case["f"]), R=om.e_in(case["R"]), g=case["g"],
                     theta=case["theta"], nsub=case["nsub"], tau=case["tau"])
    refs = [om.v_out(ref[0]), om.e_out(ref[1]), om.e_out(ref[2]), om.v_out(ref[3])]
    # the mesh's default plan, then 256,5,512 (three triangles per thread in FP64)
    for plan in (None, (256, 5, 512)):
        if plan is not None:
            assert mesh.plan_stats(*plan)["tri_per_thread"] == 3
            mesh.set_plan(*plan)
        g = mesh.adjoint(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"],
                         dt=case["tau"], params=p, ckpt_every=case["ckpt_every"], lam_eta=lam)
        outs = [mesh.v_out(g[0].cpu().numpy()), mesh.e_out(g[1].cpu().numpy()),
                mesh.e_out(g[2].cpu().numpy()), mesh.v_out(g[3].cpu().numpy())]
        for a, b in zip(outs, refs):
            assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), plan


def test_c4_ensemble_members_equal_oracle_10_steps():
    from paper_2311_08241_amd import Batch, Mesh, Params, batch_inputs
    cases = sesynth.batch_c4()
    meshes = [Mesh.from_dict(c, device=0) for c in cases]
    batch = Batch(meshes)
    nsub = [c["nsub"] for c in cases]
    # FP32 at the ensemble's shipped plan; FP64 at the first plan of a shortlist that fits
    plans = {"f32": (448, 4, 512)}
    for pl in [(448, 4, 512), (352, 4, 512), (256, 4, 256), (128, 2, 256)]:
        if batch.plan_stats(*pl)["ok_f64"]:
            plans["f64"] = pl
            break
    assert batch.plan_stats(*plans["f32"])["ok_f32"] and "f64" in plans
    dts = [c["tau"] for c in cases]
    eta_ref = float(np.mean(np.concatenate([c["eta0"] for c in cases])))
    res = {}
    for prec in ("f32", "f64"):
        batch.set_plan(*plans[prec])
        p = Params(precision=prec, eta_ref=eta_ref if prec == "f32" else 0.0)
        d = batch_inputs(batch, cases, p)
        Uavg = torch.empty((batch.ne, 2), dtype=torch.float64, device="cuda:0")
        ws = batch.workspace(p, nsub)
        for _ in range(10):
            batch.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=nsub, dt=dts,
                           params=p, Uavg=Uavg, workspace=ws)
        torch.cuda.synchronize()
        assert batch.check_faults() == 0
        res[prec] = (d["eta"].double().cpu().numpy() + p.eta_ref, Uavg.cpu().numpy())
        del d, ws, Uavg
    vo, eo = batch.vert_offset, batch.elem_offset
    worst = 0.0
    for i, (m, c) in enumerate(zip(meshes, cases)):
        r = oracle.run_case(c, nsteps=10, threads=0)
        om = r["mesh"]
        eta_r, ua_r = om.v_out(r["eta"]), om.e_out(r["Uavg"])
        e64 = m.v_out(res["f64"][0][vo[i]:vo[i + 1]])
        u64 = m.e_out(res["f64"][1][eo[i]:eo[i + 1]])
        assert np.abs(e64 - eta_r).max() <= 1e-12 * np.abs(eta_r).max(), i
        assert np.abs(u64 - ua_r).max() <= 1e-12 * np.abs(ua_r).max(), i
        e32 = m.v_out(res["f32"][0][vo[i]:vo[i + 1]])
        u32 = m.e_out(res["f32"][1][eo[i]:eo[i + 1]])
        e = np.abs(e32 - eta_r).max() / np.abs(eta_r - eta_ref).max()
        u = np.abs(u32 - ua_r).max() / np.abs(ua_r).max()
        worst = max(worst, e)
        assert e <= 1e-5, (i, nsub[i] * 10, e)
        assert u <= 1e-5, (i, nsub[i] * 10, u)
    print(f"ensemble FP32 worst member eta e_max {worst:.2e}", flush=True)


def _sesm_gpu(mesh, case, prec, plan, nsteps):
    from paper_2311_08241_amd import Params, device_inputs
    from paper_2311_08241_amd.api import sesm_coefficients
    mesh.set_plan(*plan)
    p = Params(precision=prec, eta_ref=case["eta_ref"] if prec == "f32" else 0.0, scheme="sesm",
               sesm=sesm_coefficients(case["theta"]))
    d = device_inputs(mesh, case, p)
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    ws = mesh.workspace(p, case["nsub"])
    for _ in range(nsteps):
        mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"],
                      dt=case["tau"], params=p, Uavg=Uavg, workspace=ws)
    torch.cuda.synchronize()
    assert mesh.check_faults() == 0
    eta = d["eta"].double().cpu().numpy() + p.eta_ref
    return mesh.v_out(eta), mesh.e_out(Uavg.cpu().numpy())


def _sesm_oracle(om, case, nsteps):
    from oracle import analytic
    b, d, g, z = analytic.sesm_params(case["theta"])
    H0, f, R = om.v_in(case["H0"]), om.e_in(case["f"]), om.e_in(case["R"])
    eta, U = om.v_in(case["eta0"]), om.e_in(case["U0"])
    for _ in range(nsteps):
        eta, U, Uavg, _ = om.subcycle_sesm(eta, U, H0=H0, f=f, R=R, g=case["g"], beta=b, delta=d,
                                           gamma=g, zeta=z, nsub=case["nsub"], tau=case["tau"],
                                           volume=False)
    return om.v_out(eta), om.e_out(Uavg)


def test_c3_sesm_fp64_one_step_equals_oracle():
    case, mesh, om = _c3()
    eta_r, ua_r = _sesm_oracle(om, case, 1)
    eta, ua = _sesm_gpu(mesh, case, "f64", (384, 4, 512), 1)
    assert np.abs(eta - eta_r).max() <= 1e-12 * np.abs(eta_r).max()
    assert np.abs(ua - ua_r).max() <= 1e-12 * np.abs(ua_r).max()


def test_c2_sesm_fp32_1020_substep_budget():
    from paper_2311_08241_amd import Mesh
    case = sesynth.channel_c2(nsteps=17)
    mesh = Mesh.from_dict(case, device=0)
    om = oracle.Mesh(case, reordered=True)
    eta, ua = _sesm_gpu(mesh, case, "f32", (448, 4, 512), 17)
    eta_r, ua_r = _sesm_oracle(om, case, 17)
    e_max = np.abs(eta - eta_r).max() / np.abs(eta_r - case["eta_ref"]).max()
    assert e_max <= 1e-5, e_max


def test_c3_forcing_40_layers_matches_oracle():
    """Vertically integrated forcing on the lat-lon mesh, 40 layers following the
    bathymetry, in the launch the benchmark times; bar as in test_gpu_forcing."""
    case, mesh, _ = _c3()
    K = 40
    d = sesynth.column_forcing(case, K=K, seed=0)
    dev = {k: torch.tensor(d[k], dtype=torch.float64, device="cuda:0")
           for k in ("RA", "RP", "RhV", "tau_s", "u")}
    nlev = torch.tensor(d["nlev"], dtype=torch.int32, device="cuda:0")
    R = mesh.forcing(K=K, nlev=nlev, Cd=d["Cd"], **dev)
    torch.cuda.synchronize()
    R = R.cpu().numpy()
    del dev
    ref = oracle.forcing(K=K, nlev=d["nlev"], RA=d["RA"], RP=d["RP"], RhV=d["RhV"],
                         tau_s=d["tau_s"], u=d["u"], Cd=d["Cd"])
    n = d["nlev"]
    act = (np.arange(K)[None, :] < n[:, None])[:, :, None]
    S = sum(np.where(act, np.abs(d[k]), 0.0).sum(axis=1) for k in ("RA", "RP", "RhV"))
    ub = d["u"][np.arange(n.size), n - 1]
    S = S + np.abs(d["tau_s"]) + d["Cd"] * np.hypot(ub[:, 0], ub[:, 1])[:, None] * np.abs(ub)
    assert np.all(np.abs(R - ref) <= 2.0 * (3 * n[:, None] + 6) * 2.0 ** -53 * S)
    assert mesh.check_faults() == 0


def test_c3_trim_zstar_40_layers_matches_oracle():
    """Trim/z* consumer on the lat-lon mesh at 40 layers (the benchmark's launch);
    1e-12 relative as in test_gpu_trim."""
    case, mesh, om = _c3()
    K = 40
    r = sesynth.rng(55)
    H0 = om.v_in(case["H0"])
    eta0 = om.v_in(case["eta0"])
    eta_new = eta0 + 0.01 * r.standard_normal(eta0.size)
    Uavg = r.standard_normal((om.ne, 2))
    lay = sesynth.layers(case, K=K, seed=0)
    Ustar = np.ascontiguousarray(lay["Ustar"][om.eperm])
    h0 = H0[:, None] * lay["frac"][None, :]
    hn = h0 * ((H0 + eta0) / H0)[:, None]
    tau = case["tau"]
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda:0")
    U, hnew, w = mesh.trim_zstar(H0=t(H0), eta_new=t(eta_new), Uavg=t(Uavg), Ustar=t(Ustar),
                                 hn=t(hn), h0=t(h0), tau=tau)
    torch.cuda.synchronize()
    out = (U.cpu().numpy(), hnew.cpu().numpy(), w.cpu().numpy())
    del U, hnew, w
    ref = om.trim_zstar(H0=H0, eta_new=eta_new, Uavg=Uavg, Ustar=Ustar, hn=hn, h0=h0, tau=tau)
    for a, b in zip(out, ref):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
