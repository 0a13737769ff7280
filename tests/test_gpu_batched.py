"""Batched ensemble (se_subcycle_batched) against the oracle and against
standalone member runs.

Each member of an ensemble is an independent subcycle (Sec. 2.2, eq. (eq4_10),
with the averaged transport of eq. (eq4_12)), so every member's elevation,
transport, averaged transport and volume are compared with the oracle run on
that member alone: FP64 within 1e-12, FP32 within 1e-5 after at least 1000
substeps.  With the same plan the batched launch also evaluates exactly the
operations of each member's own se_subcycle, so results must be bit-identical
to standalone runs in both precisions.  Graph replays are checked against
eager execution, with eager work and synchronisations between the replays.
"""
import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _members(n=5, seed=0):
    cases = sesynth.batch_c4(seed=seed, nmembers=n, nv_lo=800, nv_hi=6000, m_lo=5, m_hi=23)
    return cases


def _setup(cases, precision, plan=(256, 4, 512)):
    from paper_2311_08241_amd import Batch, Mesh, Params
    meshes = [Mesh.from_dict(c, device=0) for c in cases]
    for m in meshes:
        m.set_plan(*plan)
    batch = Batch(meshes)
    batch.set_plan(*plan)
    eta_ref = float(np.mean(np.concatenate([c["eta0"] for c in cases]))) if precision == "f32" else 0.0
    params = Params(g=9.81, theta=0.14, precision=precision, eta_ref=eta_ref)
    return batch, meshes, params


def _standalone(mesh, case, params):
    from paper_2311_08241_amd import device_inputs
    d = device_inputs(mesh, case, params)
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    vol = torch.empty(case["nsub"] + 1, dtype=torch.float64, device="cuda:0")
    mesh.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"],
                  dt=case["tau"], params=params, Uavg=Uavg, volume=vol)
    return d["eta"], d["U"], Uavg, vol


def _batched(batch, cases, params, use_graph=False, stream=None, d=None, ws=None):
    from paper_2311_08241_amd import batch_inputs
    d = d or batch_inputs(batch, cases, params)
    nsub = [c["nsub"] for c in cases]
    dt = [c["tau"] for c in cases]
    Uavg = torch.empty((batch.ne, 2), dtype=torch.float64, device="cuda:0")
    vol = torch.empty(batch.volume_size(params, nsub), dtype=torch.float64, device="cuda:0")
    batch.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=nsub, dt=dt,
                   params=params, Uavg=Uavg, volume=vol, use_graph=use_graph, stream=stream,
                   workspace=ws)
    return d, Uavg, vol


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("plan", [(256, 4, 512), (128, 3, 256)])
def test_batched_equals_standalone(precision, plan):
    cases = _members()
    batch, meshes, params = _setup(cases, precision, plan)
    d, Uavg, vol = _batched(batch, cases, params)
    torch.cuda.synchronize()
    assert batch.check_faults() == 0
    vo, eo = batch.vert_offset, batch.elem_offset
    voff = 0
    for i, (m, c) in enumerate(zip(meshes, cases)):
        e1, U1, ua1, v1 = _standalone(m, c, params)
        torch.cuda.synchronize()
        assert torch.equal(d["eta"][vo[i]:vo[i + 1]], e1)
        assert torch.equal(d["U"][eo[i]:eo[i + 1]], U1)
        assert torch.equal(Uavg[eo[i]:eo[i + 1]], ua1)
        n = c["nsub"] + 1
        assert torch.allclose(vol[voff:voff + n], v1, rtol=1e-14, atol=0)
        voff += n


def test_graph_replays_match_eager():
    cases = _members(4, seed=1)
    batch, meshes, params = _setup(cases, "f32", (256, 4, 512))
    from paper_2311_08241_amd import batch_inputs
    base = batch_inputs(batch, cases, params)
    nsub = [c["nsub"] for c in cases]
    s = torch.cuda.Stream()
    ws = batch.workspace(params, nsub)
    # eager reference: three chained steps
    ref = {k: (v.clone() if v is not None else None) for k, v in base.items()}
    outs = []
    with torch.cuda.stream(s):
        for _ in range(3):
            _, ua, vol = _batched(batch, cases, params, use_graph=False, stream=s, d=ref, ws=ws)
            outs.append((ref["eta"].clone(), ua.clone(), vol.clone()))
    s.synchronize()
    # graph: same chain, eager work and syncs in between
    g = {k: (v.clone() if v is not None else None) for k, v in base.items()}
    Uavg = torch.empty((batch.ne, 2), dtype=torch.float64, device="cuda:0")
    vol = torch.empty(batch.volume_size(params, nsub), dtype=torch.float64, device="cuda:0")
    with torch.cuda.stream(s):
        for k in range(3):
            batch.subcycle(g["eta"], g["U"], R=g["R"], f=g["f"], H0=g["H0"], nsub=nsub,
                           dt=[c["tau"] for c in cases], params=params, Uavg=Uavg, volume=vol,
                           use_graph=True, stream=s, workspace=ws)
            junk = torch.randn(1000, device="cuda:0") * 2   # unrelated eager work
            s.synchronize()
            assert torch.equal(g["eta"], outs[k][0])
            assert torch.equal(Uavg, outs[k][1])
            assert torch.equal(vol, outs[k][2])
    assert batch.check_faults(stream=s) == 0
    del junk


def test_batch_argument_errors():
    from paper_2311_08241_amd import _lib as L
    cases = _members(2, seed=2)
    batch, meshes, params = _setup(cases, "f64")
    d, _, _ = _batched(batch, cases, params)
    with pytest.raises(L.SeError):
        batch.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=[5, 0],
                       dt=[10.0, 10.0], params=params)
    with pytest.raises(L.SeError):      # graph capture on the default stream
        batch.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=[5, 5],
                       dt=[10.0, 10.0], params=params, use_graph=True)


# five basins of 10k-200k vertices, each with its own substep count (84-120) and
# substep length; 12 calls give every member 1008-1440 substeps
_ORC = {}


def _oracle_members(cases, ncalls):
    key = (id(cases[0]), ncalls)
    if key not in _ORC:
        out = []
        for c in cases:
            m = oracle.Mesh(c, reordered=True)
            r = oracle.run_case(c, nsteps=ncalls, mesh=m, threads=0)
            nvol = c["nsub"] + 1
            out.append((m.v_out(r["eta"]), m.e_out(r["U"]), m.e_out(r["Uavg"]),
                        r["volume"][-nvol:], m.v_out(m.Av)))
        _ORC.clear()
        _ORC[key] = out
    return _ORC[key]


_C4_PARITY = {}


def _parity_members():
    if "cases" not in _C4_PARITY:
        _C4_PARITY["cases"] = sesynth.batch_c4(seed=3, nmembers=5, m_lo=84, m_hi=120)
    return _C4_PARITY["cases"]


@pytest.mark.parametrize("precision,plan", [("f64", (352, 4, 512)), ("f32", (352, 4, 512)),
                                            ("f32", (448, 4, 512))])
def test_batched_members_equal_oracle_after_1000_substeps(precision, plan):
    from paper_2311_08241_amd import Batch, Mesh, Params, batch_inputs
    cases = _parity_members()
    ncalls = 12
    assert all(10_000 <= c["x"].size <= 200_000 for c in cases)
    assert min(c["nsub"] for c in cases) * ncalls >= 1000
    assert len({c["nsub"] for c in cases}) > 1 and len({c["tau"] / c["nsub"] for c in cases}) > 1
    meshes = [Mesh.from_dict(c, device=0) for c in cases]
    batch = Batch(meshes)
    batch.set_plan(*plan)
    eta_ref = float(np.mean(np.concatenate([c["eta0"] for c in cases])))
    p = Params(precision=precision, eta_ref=eta_ref if precision == "f32" else 0.0)
    d = batch_inputs(batch, cases, p)
    nsub = [c["nsub"] for c in cases]
    dts = [c["tau"] for c in cases]
    Uavg = torch.empty((batch.ne, 2), dtype=torch.float64, device="cuda:0")
    vol = torch.empty(batch.volume_size(p, nsub), dtype=torch.float64, device="cuda:0")
    ws = batch.workspace(p, nsub)
    for _ in range(ncalls):
        batch.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=nsub, dt=dts,
                       params=p, Uavg=Uavg, volume=vol, workspace=ws)
    torch.cuda.synchronize()
    assert batch.check_faults() == 0
    eta = d["eta"].double().cpu().numpy() + p.eta_ref
    U = d["U"].double().cpu().numpy()
    ua, vol = Uavg.cpu().numpy(), vol.cpu().numpy()
    ref = _oracle_members(cases, ncalls)
    vo, eo = batch.vert_offset, batch.elem_offset
    voff = 0
    for i, (m, c) in enumerate(zip(meshes, cases)):
        eta_r, U_r, ua_r, vol_r, Av = ref[i]
        e_i = m.v_out(eta[vo[i]:vo[i + 1]])
        u_i = m.e_out(U[eo[i]:eo[i + 1]])
        a_i = m.e_out(ua[eo[i]:eo[i + 1]])
        n = c["nsub"] + 1
        v_i = vol[voff:voff + n]
        voff += n
        if precision == "f64":
            tol = 1e-12
            assert np.abs(e_i - eta_r).max() <= tol * np.abs(eta_r).max(), i
            assert np.abs(u_i - U_r).max() <= tol * np.abs(U_r).max(), i
            assert np.abs(a_i - ua_r).max() <= tol * np.abs(ua_r).max(), i
            scale = np.sum(Av * np.abs(eta_r))
            assert np.abs(v_i - vol_r).max() <= tol * scale, i
        else:
            den = np.abs(eta_r - eta_ref).max()
            e_max = np.abs(e_i - eta_r).max() / den
            e_rms = np.sqrt(np.sum(Av * (e_i - eta_r) ** 2) / np.sum(Av * (eta_r - eta_ref) ** 2))
            u_max = np.abs(a_i - ua_r).max() / np.abs(ua_r).max()
            print(f"member {i}: nv {m.nv} nsub {c['nsub']} x {ncalls}: eta e_max {e_max:.2e} "
                  f"e_rms {e_rms:.2e}, <<U>> e_max {u_max:.2e}", flush=True)
            assert e_max <= 1e-5, (i, e_max)
            assert u_max <= 1e-5, (i, u_max)
            assert np.abs(v_i - vol_r).max() <= 1e-5 * Av.sum() * den, i
