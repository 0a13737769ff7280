"""Batched ensemble (se_subcycle_batched) against standalone member runs.

With the same plan the batched launch evaluates exactly the operations of
each member's own se_subcycle, so results must be bit-identical in both
precisions; the FP64 member runs are themselves equal to the oracle (see the
forward tests).  Graph replays are checked against eager execution, with
eager work and synchronisations between the replays.
"""
import numpy as np
import pytest

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
