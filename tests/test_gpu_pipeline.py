"""The barotropic part of one baroclinic step end to end on the GPU, against the same
chain in the FP64 oracle:

  vertically integrated forcing R (eq. (eq4_4)) from synthetic layers
  -> subcycle with the barotropic viscous term (eq. (eq4_10), eq. (eq:viscosity_BT);
     tile kernel and plain path)
  -> trim of the layer transports to <<U>> and z* thicknesses (eq. (eq4_13), Sec. 2.4)

Bars: 1e-12 relative for the subcycle and trim outputs (the forcing differs from the
oracle's only in summation order); the column closes (surface w ~ 0) on the GPU.
"""
import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("plain", [True, False])
def test_forcing_subcycle_trim_chain(plain):
    from paper_2311_08241_amd import Mesh, Params, device_inputs
    case = sesynth.channel_c2(nx=128, ny=64, nsteps=1)
    K = 30
    col = sesynth.column_forcing(case, K=K, seed=4)
    om = oracle.Mesh(case, reordered=True)
    mesh = Mesh.from_dict(case, device=0)
    assert np.array_equal(mesh.eperm, om.eperm) and np.array_equal(mesh.vperm, om.vperm)
    e_in = lambda a: np.ascontiguousarray(np.asarray(a)[om.eperm])
    t = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda:0")

    # 1. forcing
    R_o = oracle.forcing(K=K, nlev=e_in(col["nlev"]), RA=e_in(col["RA"]), RP=e_in(col["RP"]),
                         RhV=e_in(col["RhV"]), tau_s=e_in(col["tau_s"]), u=e_in(col["u"]),
                         Cd=col["Cd"])
    R_g = mesh.forcing(K=K, nlev=t(e_in(col["nlev"]), torch.int32), RA=t(e_in(col["RA"])),
                       RP=t(e_in(col["RP"])), RhV=t(e_in(col["RhV"])),
                       tau_s=t(e_in(col["tau_s"])), u=t(e_in(col["u"])), Cd=col["Cd"])
    assert _rel(R_g.cpu().numpy(), R_o) <= 1e-12

    # 2. subcycle with the viscous term, R from step 1 on each side
    visc = (200.0, 0.1)
    H0, eta0 = om.v_in(case["H0"]), om.v_in(case["eta0"])
    eta_o, U_o, Uavg_o, _ = om.subcycle(eta0, om.e_in(case["U0"]), H0=H0, f=om.e_in(case["f"]),
                                        R=R_o, g=case["g"], theta=case["theta"],
                                        nsub=case["nsub"], tau=case["tau"], visc=visc)
    p = Params(g=case["g"], theta=case["theta"], precision="f64", visc=visc)
    if not plain:
        mesh.set_plan(128, 4, 256)
    d = device_inputs(mesh, case, p)
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    mesh.subcycle(d["eta"], d["U"], R=R_g, f=d["f"], H0=d["H0"], nsub=case["nsub"],
                  dt=case["tau"], params=p, Uavg=Uavg, workspace=mesh.workspace(p, case["nsub"]),
                  plain=plain)
    torch.cuda.synchronize()
    assert mesh.check_faults() == 0
    assert _rel(d["eta"].cpu().numpy(), eta_o) <= 1e-12
    assert _rel(Uavg.cpu().numpy(), Uavg_o) <= 1e-12

    # 3. trim and z* from the subcycle's outputs
    lay = sesynth.layers(case, K=K, seed=2)
    Ustar = e_in(lay["Ustar"])
    h0 = H0[:, None] * lay["frac"][None, :]
    hn = h0 * ((H0 + eta0) / H0)[:, None]
    ref = om.trim_zstar(H0=H0, eta_new=eta_o, Uavg=Uavg_o, Ustar=Ustar, hn=hn, h0=h0,
                        tau=case["tau"])
    U, hnew, w = mesh.trim_zstar(H0=d["H0"], eta_new=d["eta"], Uavg=Uavg, Ustar=t(Ustar),
                                 hn=t(hn), h0=t(h0), tau=case["tau"])
    torch.cuda.synchronize()
    out = (U.cpu().numpy(), hnew.cpu().numpy(), w.cpu().numpy())
    for a, b in zip(out, ref):
        assert _rel(a, b) <= 1e-12
    # the column closes: layer sums equal <<U>>, the surface velocity vanishes
    assert _rel(out[0].sum(1), Uavg_o) <= 1e-12
    assert np.abs(out[2][:, 0]).max() <= 1e-12 * H0.max() / case["tau"]
