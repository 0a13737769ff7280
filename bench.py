"""Benchmark of the barotropic subcycle on one MI355X.

A step is one baroclinic step of the global-scale lat-lon workload: 80
dissipative forward-backward substeps on the 2048 x 1536 lat-lon mesh with a
30% land mask (about 2.2M wet vertices, 4.3M triangles), FP32 bulk with FP64
volume and averaged transport, followed by the averaged transport.  Inputs are
seeded and synthetic and resident in HBM before timing starts.

Prints one JSON line with: throughput in vertex-substeps/s, the roofline
position of the dominant kernel (its compulsory bytes per launch -- one pass
over the state, forcing, geometry, connectivity and running sums, 236 B per
vertex in FP32 -- over the average launch time, against 8 TB/s), the plain
FP64 GPU path and the FP64 fused path on the same workload, errors of the
timed configuration against the FP64 oracle after 13 steps (1040 substeps),
and the oracle timed on this host's cores (all cores, and one thread).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("vertex-substeps/s + HBM GB/s, FP32/batched vs FP64 plain at stated η error")
HBM_PEAK_GBS = 8000.0
# Compulsory bytes per vertex of one streaming pass over everything a substep
# touches (r = triangles per vertex ~ 2):
#   vertex: eta r+w, H0, 1/A_v, row pointer; triangle: U r+w, R, f, geometry,
#   connectivity, running sum r+w, CSR column.
# The tile kernel makes one such pass per launch of k substeps (the state stays on
# chip in between), so its compulsory traffic per launch is B_ALG x nv.
B_ALG = {"f32": 236.0, "f64": 356.0}
# baroclinic steps (13 x 80 = 1040 substeps) after which the errors of the timed
# configuration are measured against the oracle
ERR_STEPS = 13


def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SUBCYCLE_SOURCES = ("kernels.hip", "kernels.h", "device_common.h")


def kernel_source_hash():
    """Hash of the subcycle kernels' sources (the tile kernel and what it includes)."""
    h = hashlib.sha256()
    for name in SUBCYCLE_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_08241_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload_tag, plan):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken with the same kernel source and plan."""
    path = os.path.join(ROOT, "profiles", f"pmc_k_tile_{workload_tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("subcycle_sources_sha256_16") != kernel_source_hash():
        return None
    if kv.get("plan") != ",".join(str(v) for v in plan):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _time(fn, n, stream=None):
    import torch
    s = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def bench_batched(args, log, with_oracle=True):
    """Ensemble of 64 jittered basins (10k-200k vertices, 20-120 substeps): one graph-captured
    FP32 batched launch sequence vs a per-member loop of the plain FP64 path; both against
    the FP64 oracle, member by member."""
    import torch

    import sesynth
    from paper_2311_08241_amd import Batch, Mesh, Params, batch_inputs, device_inputs
    from paper_2311_08241_amd.autotune import autotune
    t0 = time.time()
    cases = sesynth.batch_c4() if not args.small else sesynth.batch_c4(nmembers=8, nv_hi=30000)
    meshes = [Mesh.from_dict(c, device=0) for c in cases]
    batch = Batch(meshes)
    nsub = [c["nsub"] for c in cases]
    dts = [c["tau"] for c in cases]
    work = float(sum(m.nv * k for m, k in zip(meshes, nsub)))
    log(f"[bench] ensemble: {len(cases)} members, {batch.nv} vertices, "
        f"{work:.3e} vertex-substeps per step ({time.time() - t0:.1f}s setup)")
    eta_ref = float(np.mean(np.concatenate([c["eta0"] for c in cases])))
    p32 = Params(precision="f32", eta_ref=eta_ref, track_volume=True)
    p64 = Params(precision="f64", track_volume=True)
    d32 = batch_inputs(batch, cases, p32)
    stream = torch.cuda.Stream()
    ws = batch.workspace(p32, nsub)
    Uavg = torch.empty((batch.ne, 2), dtype=torch.float64, device="cuda:0")
    vol = torch.empty(batch.volume_size(p32, nsub), dtype=torch.float64, device="cuda:0")
    e_init, u_init = d32["eta"].clone(), d32["U"].clone()

    def reset():
        d32["eta"].copy_(e_init)
        d32["U"].copy_(u_init)

    def step(graph=True):
        batch.subcycle(d32["eta"], d32["U"], R=d32["R"], f=d32["f"], H0=d32["H0"], nsub=nsub,
                       dt=dts, params=p32, Uavg=Uavg, volume=vol, workspace=ws,
                       use_graph=graph, stream=stream)
    with torch.cuda.stream(stream):
        tune = autotune(batch, lambda: step(False), "f32", max(nsub), top=24, log=log,
                        reset=reset, use_cache=not args.retune)
        reset()
        step(True)          # capture
        stream.synchronize()
        reset()
        step(True)
        stream.synchronize()
        eta32 = d32["eta"].double().cpu().numpy() + eta_ref
        ua32 = Uavg.cpu().numpy()
        ms = _time(lambda: step(True), 5, stream)
    faults = batch.check_faults(stream=stream)
    log(f"[bench] ensemble FP32 batched (graph): {ms:.2f} ms/step, {work / ms * 1e3:.3e} "
        f"vertex-substeps/s, plan {tune['plan']}")
    # FP64 reference and baseline: per-member loop of the plain path
    members64 = []
    for m, c in zip(meshes, cases):
        d = device_inputs(m, c, p64)
        members64.append((m, c, d, torch.empty((m.ne, 2), dtype=torch.float64, device="cuda:0"),
                          m.workspace(p64, c["nsub"]), d["eta"].clone(), d["U"].clone()))

    def loop64():
        for m, c, d, ua, w, _, _ in members64:
            m.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=c["nsub"],
                       dt=c["tau"], params=p64, Uavg=ua, workspace=w, plain=True)
    loop64()
    torch.cuda.synchronize()
    # errors of one step (M_i substeps per member) against the oracle (all host cores)
    err = {"eta_max": 0.0, "Uavg_max": 0.0, "fp64_eta_max": 0.0, "fp64_Uavg_max": 0.0}
    vo, eo = batch.vert_offset, batch.elem_offset
    t0 = time.perf_counter()
    if with_oracle:
        import oracle
    for i, (m, c, d, ua, w, e0_, u0_) in enumerate(members64):
        e64 = m.v_out(d["eta"].cpu().numpy())
        ua64 = m.e_out(ua.cpu().numpy())
        d["eta"].copy_(e0_)
        d["U"].copy_(u0_)
        if not with_oracle:
            continue
        ref = oracle.run_case(c, nsteps=1, threads=0)
        om = ref["mesh"]
        eta_r, ua_r = om.v_out(ref["eta"]), om.e_out(ref["Uavg"])
        den, uden = np.abs(eta_r - eta_ref).max(), np.abs(ua_r).max()
        e32 = m.v_out(eta32[vo[i]:vo[i + 1]])
        u32 = m.e_out(ua32[eo[i]:eo[i + 1]])
        err["eta_max"] = max(err["eta_max"], float(np.abs(e32 - eta_r).max() / den))
        err["Uavg_max"] = max(err["Uavg_max"], float(np.abs(u32 - ua_r).max() / uden))
        err["fp64_eta_max"] = max(err["fp64_eta_max"], float(np.abs(e64 - eta_r).max() /
                                                             np.abs(eta_r).max()))
        err["fp64_Uavg_max"] = max(err["fp64_Uavg_max"], float(np.abs(ua64 - ua_r).max() / uden))
    if with_oracle:
        log(f"[bench] ensemble errors vs oracle ({time.perf_counter() - t0:.1f} s): {err}")
    ms64 = _time(loop64, 2)
    log(f"[bench] ensemble FP64 per-member plain loop: {ms64:.2f} ms/step")
    return {"workload": f"{len(cases)} jittered basins, {batch.nv} vertices, substeps "
                        f"{min(nsub)}-{max(nsub)}",
            "value": work / ms * 1e3, "unit": "vertex-substeps/s", "ms_per_step": ms,
            "plan": tune["plan"], "graph": True, "faults": faults,
            "fp64_member_loop": {"value": work / ms64 * 1e3, "ms_per_step": ms64},
            "speedup_vs_fp64_member_loop": ms64 / ms,
            "errors_vs_oracle": (dict(err, after="one step (M_i substeps) per member")
                                 if with_oracle else None)}


def bench_adjoint(args, log):
    """Adjoint workload: 256x256 jittered basin, 30 substeps, checkpoints every 5."""
    import torch

    import sesynth
    from paper_2311_08241_amd import Mesh, Params, device_inputs
    case = sesynth.adjoint_c5()
    mesh = Mesh.from_dict(case, device=0)
    out = {"workload": f"{mesh.nv} vertices, {case['nsub']} substeps, checkpoint every "
                       f"{case['ckpt_every']}"}
    for prec in ("f64", "f32"):
        p = Params(precision=prec, eta_ref=case["eta_ref"] if prec == "f32" else 0.0)
        d = device_inputs(mesh, case, p)
        lam = torch.ones(mesh.nv, dtype=p.dtype, device="cuda:0")
        g = [torch.empty_like(d["eta"]), torch.empty_like(d["U"]), torch.empty_like(d["R"]),
             torch.empty_like(d["H0"])]
        e, U = d["eta"].clone(), d["U"].clone()
        ws = None

        def fwd():
            mesh.subcycle(e, U, R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"],
                          dt=case["tau"], params=p, workspace=ws)

        def adj():
            mesh.adjoint(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=case["nsub"],
                         dt=case["tau"], params=p, ckpt_every=case["ckpt_every"], lam_eta=lam,
                         g_eta0=g[0], g_U0=g[1], g_R=g[2], g_H0=g[3], workspace=ws)

        def use(plan):
            nonlocal ws
            mesh.set_plan(*plan)
            ws = mesh.workspace(p, case["nsub"], case["ckpt_every"])
        # tile plans for this mesh (shapes that give 64-512 tiles, with 2-6 substeps per
        # launch; 5 or more run a checkpoint segment in one launch): the forward and the
        # adjoint are each timed on every plan and each is reported at its fastest
        bestf = besta = None
        for plan in ((1024, 4, 512), (512, 4, 512), (256, 4, 256), (128, 4, 256),
                     (256, 5, 256), (128, 5, 256), (128, 6, 256), (256, 5, 512),
                     (192, 5, 512), (320, 5, 512), (128, 5, 512), (256, 5, 1024)):
            if not mesh.plan_stats(*plan)["ok_f32" if prec == "f32" else "ok_f64"]:
                continue
            use(plan)
            fwd()
            t = _time(fwd, 5)
            if bestf is None or t < bestf[0]:
                bestf = (t, plan)
            adj()
            ta = _time(adj, 5)
            log(f"[bench] adjoint {prec} plan {plan}: forward {t:.3f} ms, adjoint {ta:.3f} ms")
            if besta is None or ta < besta[0]:
                besta = (ta, plan)
        use(besta[1])
        adj()
        torch.cuda.synchronize()
        ms = _time(adj, 5)
        # the same call captured in a graph (kernels and device copies only): launch
        # overhead dominates at this size
        ref = [x.clone() for x in g]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            adj()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            adj()
        graph.replay()
        torch.cuda.synchronize()
        if not all(torch.equal(a, b) for a, b in zip(g, ref)):
            raise RuntimeError("adjoint graph replay differs from the eager gradients")
        ms_graph = _time(graph.replay, 10)
        use(bestf[1])
        fwd()
        msf = _time(fwd, 5)
        # launches in stream order, each waiting for the previous one (the tile path of
        # se_subcycle_adjoint): the sweep up to the last checkpoint, ceil(k / k_fused)
        # tile launches per segment; the last segment's recompute; per segment its
        # reverse launches (ceil(len / k_fused)), the recompute of the segment before it
        # sharing them (the first reverse launch starts from the seeds, the last one
        # writes the gradients of the initial state)
        nsub, k = case["nsub"], case["ckpt_every"]
        K = besta[1][1]
        segs = [min(k, nsub - m0) for m0 in range(0, nsub, k)]
        nch = lambda L: -(-L // K)
        rec = lambda L: nch(L) if L > 1 else 0
        nops = (nch(k) * (len(segs) - 1) + rec(segs[-1])
                + sum(max(nch(L), rec(segs[i - 1]) if i > 0 else 0) for i, L in enumerate(segs)))
        out[prec] = {"plan": list(besta[1]), "forward_plan": list(bestf[1]),
                     "ms_adjoint": ms, "ms_adjoint_graph": ms_graph, "ms_forward": msf,
                     "adjoint_over_forward": ms / msf, "dependent_launches": nops,
                     "us_per_launch": 1e3 * ms_graph / nops}
        log(f"[bench] adjoint {prec}: {ms:.3f} ms at {besta[1]}, graph replay {ms_graph:.3f} ms "
            f"(forward {msf:.3f} ms at {bestf[1]}; {nops} dependent launches, "
            f"{1e3 * ms_graph / nops:.1f} us each)")
    return out


def bench_share(args, log, mesh, case, value_full, nparts=8):
    """One GPU's share of the lat-lon workload at its real size: a contiguous 1/nparts
    range of the library's Hilbert vertex order (the middle one), as a mesh of its own
    whose cut edge is a coast instead of a halo, FP32, the fastest of a few tile plans.
    What it leaves out: the halo exchange every k_fused substeps and the volume
    all-reduce of a multi-GPU run."""
    import torch

    import sesynth
    from paper_2311_08241_amd import Mesh, Params, device_inputs
    k = nparts // 2
    lo, hi = k * mesh.nv // nparts, (k + 1) * mesh.nv // nparts
    sub = sesynth.vertex_subset(case, mesh.vperm[lo:hi], name=f"{case['name']}-share{k}of{nparts}")
    m = Mesh.from_dict(sub, device=0)
    nsub, tau = sub["nsub"], sub["tau"]
    p = Params(g=sub["g"], theta=sub["theta"], precision="f32", eta_ref=sub["eta_ref"],
               track_volume=True)
    d = device_inputs(m, sub, p)
    Uavg = torch.empty((m.ne, 2), dtype=torch.float64, device="cuda:0")
    vol = torch.empty(nsub + 1, dtype=torch.float64, device="cuda:0")
    best = None
    for plan in ((520, 4, 512), (464, 4, 512), (384, 4, 512), (304, 4, 512), (256, 4, 512),
                 (192, 4, 512), (320, 2, 256), (256, 3, 512)):
        if not m.plan_stats(*plan)["ok_f32"]:
            continue
        m.set_plan(*plan)
        ws = m.workspace(p, nsub)

        def step():
            m.subcycle(d["eta"], d["U"], R=d["R"], f=d["f"], H0=d["H0"], nsub=nsub, dt=tau,
                       params=p, Uavg=Uavg, volume=vol, workspace=ws)
        step()
        t = _time(step, 10)
        if best is None or t < best[0]:
            best = (t, plan, m.plan_stats(*plan)["ntiles"])
    assert m.check_faults() == 0
    ms, plan, ntiles = best
    rate = m.nv * nsub / ms * 1e3
    log(f"[bench] share {k + 1}/{nparts}: {m.nv} vertices, {ms:.3f} ms/step at {plan} "
        f"({ntiles} tiles), {rate:.3e} vertex-substeps/s ({rate / value_full:.2f} of the whole mesh's)")
    return {"workload": f"vertices {lo}..{hi - 1} of the Hilbert order ({m.nv} vertices, {m.ne} "
                        f"triangles), FP32, {nsub} substeps per step",
            "plan": list(plan), "tiles": ntiles, "ms_per_step": ms, "value": rate,
            "of_whole_mesh_rate": rate / value_full}


def bench_sesm(args, log, mesh, case, stream, with_oracle):
    """The AB3-AM4 scheme (eqs. (eq4_7)-(eq4_8)) on the same lat-lon workload: FP32
    on the tile kernel (autotuned), FP64 on the plain three-kernel path, FP32 error
    against the FP64 oracle after one step."""
    import torch

    from paper_2311_08241_amd import Params, device_inputs
    from paper_2311_08241_amd.api import sesm_coefficients
    from paper_2311_08241_amd.autotune import autotune
    nsub, tau = case["nsub"], case["tau"]
    co = sesm_coefficients(case["theta"])
    out = {"coefficients": {"beta": co[0], "delta": co[1], "gamma": co[2], "zeta": co[3]}}
    p32 = Params(g=case["g"], theta=case["theta"], precision="f32", eta_ref=case["eta_ref"],
                 scheme="sesm", sesm=co)
    p64 = Params(g=case["g"], theta=case["theta"], precision="f64", scheme="sesm", sesm=co)
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    res = {}
    for label, p, plain in (("fp32_tile", p32, False), ("fp64_tile", p64, False),
                            ("fp64_plain", p64, True)):
        d = device_inputs(mesh, case, p)
        e0_, u0_ = d["eta"].clone(), d["U"].clone()
        ws = mesh.workspace(p, nsub)

        def step(dd=d, pp=p, w=ws, pl=plain):
            mesh.subcycle(dd["eta"], dd["U"], R=dd["R"], f=dd["f"], H0=dd["H0"], nsub=nsub,
                          dt=tau, params=pp, Uavg=Uavg, workspace=w, plain=pl)

        def reset(dd=d, a=e0_, b=u0_):
            dd["eta"].copy_(a)
            dd["U"].copy_(b)
        with torch.cuda.stream(stream):
            if not plain:
                key = p.precision + "-sesm"
                t = autotune(mesh, step, key, nsub, top=24 if key == "f32-sesm" else 12,
                             reps=3 if key == "f32-sesm" else 2, log=log, reset=reset,
                             use_cache=not args.retune)
                out["plan" if key == "f32-sesm" else "plan_fp64"] = t["plan"]
            reset()
            step()
            torch.cuda.synchronize()
            res[label] = (mesh.v_out(d["eta"].double().cpu().numpy() + p.eta_ref),
                          mesh.e_out(Uavg.cpu().numpy()))
            n = max(2, args.steps // 2)
            ms = _time(step, n, stream)
        out[label] = {"value": float(mesh.nv) * nsub / (ms * 1e-3), "ms_per_step": ms}
        log(f"[bench] sesm {label}: {out[label]['value']:.3e} vertex-substeps/s ({ms:.2f} ms/step)")
        del d, ws
    if mesh.check_faults():
        raise RuntimeError("kernel fault flags set (sesm)")
    if with_oracle:
        import oracle
        om = oracle.Mesh(case, reordered=True)
        b, dl, g, z = co
        t0 = time.perf_counter()
        eta_o, _, ua_o, _ = om.subcycle_sesm(om.v_in(case["eta0"]), om.e_in(case["U0"]),
                                             H0=om.v_in(case["H0"]), f=om.e_in(case["f"]),
                                             R=om.e_in(case["R"]), g=case["g"], beta=b,
                                             delta=dl, gamma=g, zeta=z, nsub=nsub, tau=tau,
                                             volume=False)
        log(f"[bench] sesm oracle step {time.perf_counter() - t0:.1f}s")
        eta_r, ua_r = om.v_out(eta_o), om.e_out(ua_o)
        for label in res:
            eta_g, ua_g = res[label]
            ref = case["eta_ref"]
            out[label]["eta_max_err"] = float(np.abs(eta_g - eta_r).max() /
                                              np.abs(eta_r - ref).max())
            out[label]["Uavg_max_err"] = float(np.abs(ua_g - ua_r).max() / np.abs(ua_r).max())
        log(f"[bench] sesm errors vs oracle: "
            f"{ {k: (out[k]['eta_max_err'], out[k]['Uavg_max_err']) for k in res} }")
    return out


def bench_trim(args, log, mesh, case, stream, K=40):
    """Consumer of <<U>> on the lat-lon mesh with K layers (FP64): trim of the layer
    transports (eq. (eq4_13)), z* thicknesses, diasurface velocity; HBM-bound, once
    per baroclinic step.  Compulsory bytes: 32 per vertex-layer (hn, h0 in; hnew,
    w out), 32 per triangle-layer (Ustar in, U out), 16 per vertex and triangle."""
    import torch

    import sesynth
    lay = sesynth.layers(case, K=K, seed=0)
    dev = "cuda:0"
    f64 = torch.float64
    H0 = torch.tensor(mesh.v_in(case["H0"]), dtype=f64, device=dev)
    eta0 = torch.tensor(mesh.v_in(case["eta0"]), dtype=f64, device=dev)
    frac = torch.tensor(lay["frac"], dtype=f64, device=dev)
    h0 = (H0[:, None] * frac[None, :]).contiguous()
    hn = (h0 * ((H0 + eta0) / H0)[:, None]).contiguous()
    Ustar = torch.tensor(np.ascontiguousarray(mesh.e_in(lay["Ustar"])), dtype=f64, device=dev)
    Uavg = Ustar.sum(1).contiguous() * 0.999
    eta_new = eta0 * 0.999
    U = torch.empty_like(Ustar)
    hnew = torch.empty_like(hn)
    w = torch.empty((mesh.nv, K + 1), dtype=f64, device=dev)

    def call():
        mesh.trim_zstar(H0=H0, eta_new=eta_new, Uavg=Uavg, Ustar=Ustar, hn=hn, h0=h0,
                        tau=case["tau"], U=U, hnew=hnew, w=w, stream=stream)
    with torch.cuda.stream(stream):
        call()
        torch.cuda.synchronize()
        ms = _time(call, 10, stream)
    nbytes = 32.0 * K * (mesh.nv + mesh.ne) + 16.0 * (mesh.nv + mesh.ne)
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"[bench] trim/z* K={K}: {ms:.3f} ms per call, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f} of peak)")
    del Ustar, U, hn, h0, hnew, w
    return {"workload": f"lat-lon mesh, {K} layers, FP64", "ms_per_call": ms,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_call": nbytes}}


def bench_visc(args, log, mesh, case, stream, visc=(2.0e3, 0.1)):
    """Barotropic viscous regularization (eq. (eq:viscosity_BT)) on the lat-lon workload:
    the subcycle carrying it on the tile kernel (two rings per substep, plan from the
    autotuner) and on the plain path (FP32 and FP64, one viscous evaluation per substep),
    and the operator alone (FP64).  Compulsory bytes of the operator per triangle: U,
    the velocity scratch written and read, base and result (16 each), neighbours 16,
    edge geometry 48, A_e 8, connectivity 12, and per vertex eta and H0 (16, about
    8 per triangle)."""
    import torch

    from paper_2311_08241_amd import Params, device_inputs
    from paper_2311_08241_amd.autotune import autotune
    nsub, tau = case["nsub"], case["tau"]
    out = {"A0": visc[0], "Cv": visc[1]}
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device="cuda:0")
    for label, prec, plain in (("fp32_tile", "f32", False), ("fp32_plain", "f32", True),
                               ("fp64_tile", "f64", False), ("fp64_plain", "f64", True)):
        p = Params(g=case["g"], theta=case["theta"], precision=prec,
                   eta_ref=case["eta_ref"] if prec == "f32" else 0.0, visc=visc)
        d = device_inputs(mesh, case, p)
        ws = mesh.workspace(p, nsub)

        def step(dd=d, pp=p, w=ws, pl=plain):
            mesh.subcycle(dd["eta"], dd["U"], R=dd["R"], f=dd["f"], H0=dd["H0"], nsub=nsub,
                          dt=tau, params=pp, Uavg=Uavg, workspace=w, plain=pl)
        with torch.cuda.stream(stream):
            if not plain:
                # plans for two rings per substep (the autotuner's viscous model)
                t = autotune(mesh, step, prec + "-visc", nsub, top=12, reps=2, final=2,
                             final_reps=4, log=log, use_cache=not args.retune)
                out[label + "_plan"] = list(t["plan"])
            step()
            torch.cuda.synchronize()
            ms = _time(step, max(2, args.steps // 4), stream)
        out[label] = {"value": float(mesh.nv) * nsub / (ms * 1e-3), "ms_per_step": ms}
        log(f"[bench] visc {label}: {out[label]['value']:.3e} vertex-substeps/s ({ms:.2f} ms/step)")
        if label == "fp64_plain":
            V = torch.empty_like(d["U"])
            scratch = torch.empty_like(d["U"])

            def op(dd=d):
                mesh.visc(dd["eta"], dd["U"], H0=dd["H0"], A0=visc[0], Cv=visc[1], V=V,
                          workspace=scratch, stream=stream)
            with torch.cuda.stream(stream):
                op()
                torch.cuda.synchronize()
                ms = _time(op, 20, stream)
            nbytes = 176.0 * mesh.ne
            gbs = nbytes / (ms * 1e-3) / 1e9
            out["operator_fp64"] = {
                "ms_per_call": ms,
                "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "bytes_per_call": nbytes}}
            log(f"[bench] visc operator fp64: {ms:.3f} ms, {gbs:.0f} GB/s")
            del V, scratch
        del d, ws
    if mesh.check_faults():
        raise RuntimeError("kernel fault flags set (viscous subcycle)")
    return out


def bench_forcing(args, log, mesh, case, stream, K=40):
    """Vertically integrated baroclinic forcing (eq. (eq4_4)) on the lat-lon mesh with
    K layers following the bathymetry (FP64 in, FP64 out); HBM-bound, once per
    baroclinic step.  Compulsory bytes: 48 per active triangle-layer (RA, RP, RhV),
    16 each for tau_s, the bottom velocity and R, 4 for the layer count."""
    import torch

    import sesynth
    d = sesynth.column_forcing(case, K=K, seed=0)
    dev = "cuda:0"
    t = {k: torch.tensor(d.pop(k), dtype=torch.float64, device=dev)
         for k in ("RA", "RP", "RhV", "u", "tau_s")}
    nlev = torch.tensor(d["nlev"], dtype=torch.int32, device=dev)
    R = torch.empty((mesh.ne, 2), dtype=torch.float64, device=dev)

    def call():
        mesh.forcing(K=K, nlev=nlev, Cd=d["Cd"], R=R, stream=stream, **t)
    with torch.cuda.stream(stream):
        call()
        torch.cuda.synchronize()
        ms = _time(call, 10, stream)
    nbytes = 48.0 * float(d["nlev"].sum()) + 52.0 * mesh.ne
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"[bench] forcing K={K}: {ms:.3f} ms per call, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f} of peak)")
    del t, R
    return {"workload": f"lat-lon mesh, {K} layers (mean {d['nlev'].mean():.1f} active), FP64",
            "ms_per_call": ms,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_call": nbytes}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--plan", default="", help="tile,k_fused,block (default: autotuned/default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP64 comparison runs")
    ap.add_argument("--small", action="store_true", help="reduced mesh (testing the script)")
    ap.add_argument("--retune", action="store_true",
                    help="time the plan candidates even if a tuned plan is cached or shipped")
    ap.add_argument("--consumers-only", action="store_true",
                    help="time only the trim/z*, forcing and viscous-term kernels (profiling)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint on the 256x256 basin (profiling)")
    ap.add_argument("--scheme", default="se", choices=["se", "sesm"],
                    help="scheme of the timed step (profiling the AB3-AM4 tile kernel)")
    ap.add_argument("--visc", default="",
                    help="A0,Cv: time the step with the barotropic viscous term (profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only (sharding over GPUs is designed "
              "but not implemented), so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import sesynth
    from paper_2311_08241_amd import Mesh, Params, device_inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.adjoint_only:
        print(json.dumps({"adjoint": bench_adjoint(args, log)}), flush=True)
        return
    t0 = time.time()
    if args.small:
        case = sesynth.latlon_c3(nlon=512, nlat=384, nsteps=args.steps)
        case["tau"] = case["nsub"] * 45.0
        tag = "C3small"
    else:
        case = sesynth.latlon_c3(nsteps=args.steps)
        tag = "C3"
    log(f"[bench] generated {case['name']}: nv={case['x'].size} ne={case['tri'].shape[0]} "
        f"in {time.time() - t0:.1f}s")
    t0 = time.time()
    mesh = Mesh.from_dict(case, device=0)
    log(f"[bench] mesh create {time.time() - t0:.1f}s, mu_max={mesh.mu_max:.3e}")
    if args.consumers_only:
        stream = torch.cuda.Stream()
        res = {"trim_zstar": bench_trim(args, log, mesh, case, stream),
               "forcing": bench_forcing(args, log, mesh, case, stream),
               "visc": bench_visc(args, log, mesh, case, stream)}
        print(json.dumps({"consumers": res, "workload": case["name"]}), flush=True)
        return
    t0 = time.time()
    nsub, tau = case["nsub"], case["tau"]
    prec = args.precision
    if args.scheme != "se" or args.visc:
        # profiling runs of the other tile-kernel forms: the timed step only
        args.no_cpu = args.no_extra = True
    variant = {}
    tune_key = prec
    if args.scheme == "sesm":
        variant["scheme"] = "sesm"
        tune_key = prec + "-sesm"
    if args.visc:
        variant["visc"] = tuple(float(v) for v in args.visc.split(","))
        tune_key = prec + "-visc"
    params = Params(g=case["g"], theta=case["theta"], precision=prec,
                    eta_ref=case["eta_ref"] if prec == "f32" else 0.0, track_volume=True,
                    **variant)
    d = device_inputs(mesh, case, params)
    Uavg = torch.empty((mesh.ne, 2), dtype=torch.float64, device=dev)
    vol = torch.empty(nsub + 1, dtype=torch.float64, device=dev)
    ws = mesh.workspace(params, nsub)

    def step(dd=d, p=params, w=ws, plain=False):
        mesh.subcycle(dd["eta"], dd["U"], R=dd["R"], f=dd["f"], H0=dd["H0"], nsub=nsub, dt=tau,
                      params=p, Uavg=Uavg, volume=vol, workspace=w, plain=plain)

    tune = None
    if args.plan:
        mesh.set_plan(*[int(v) for v in args.plan.split(",")])
    else:
        from paper_2311_08241_amd.autotune import autotune
        scratch = {k: (v.clone() if v is not None else None) for k, v in d.items()}

        def reset():
            scratch["eta"].copy_(d["eta"])
            scratch["U"].copy_(d["U"])
        tune = autotune(mesh, lambda: step(scratch), tune_key, nsub, log=log, reset=reset,
                        use_cache=not args.retune)
        del scratch
        log(f"[bench] autotuned plan {tune['plan']} ({tune['ms']:.3f} ms/step, "
            f"cached={tune['cached']})")
    plan = mesh.get_plan()

    # ERR_STEPS chained steps from the initial state at the timed plan, for the error
    # report against the oracle
    vol_0 = None
    for k in range(ERR_STEPS):
        step()
        if k == 0:
            vol_0 = float(vol[0].item())   # volume of the initial state
    torch.cuda.synchronize()
    if mesh.check_faults():
        raise RuntimeError("kernel fault flags set")
    eta_err = d["eta"].double().cpu().numpy() + (params.eta_ref if prec == "f32" else 0.0)
    Uavg_err = Uavg.cpu().numpy()
    log(f"[bench] plan tile,k,block={plan}; {ERR_STEPS} steps for the error report done "
        f"({time.time() - t0:.1f}s)")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    if mesh.check_faults():
        raise RuntimeError("kernel fault flags set")
    vsub = float(mesh.nv) * nsub * args.steps
    value = vsub / (ms * 1e-3)
    # volume drift over every step run so far (first, warm-up and timed), FP64 accumulator
    atot = float(mesh.geometry()[0].sum())
    volume_drift = {"steps": ERR_STEPS + args.warmup + args.steps,
                    "rel": abs(float(vol[-1].item()) - vol_0) /
                    (atot * float(np.abs(case["eta0"]).max()))}
    log(f"[bench] timed {args.steps} steps: {ms:.2f} ms, {value:.3e} vertex-substeps/s")

    # roofline of the dominant kernel: the tile kernel runs ceil(nsub/k) launches per
    # step, each one compulsory pass (B_ALG bytes per vertex) for k substeps
    launches_per_step = -(-nsub // (plan[1] // 2 if args.visc else plan[1]))
    avg_launch_s = ms * 1e-3 / (launches_per_step * args.steps)
    units_per_launch = float(mesh.nv)
    compulsory = B_ALG[prec] * units_per_launch
    achieved = compulsory / avg_launch_s / 1e9
    # the same bytes counted once per substep (what a kernel streaming every substep
    # from HBM would have to move for this rate)
    effective = compulsory * nsub / launches_per_step / avg_launch_s / 1e9
    traffic = None if variant else read_traffic(f"{tag}_{prec}", plan)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "k_tile",
                "unit_of_work": "vertex (one compulsory pass per launch of k substeps)",
                "bytes_per_unit": B_ALG[prec], "units_per_launch": units_per_launch,
                "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "hbm_frac_measured": (None if traffic is None else
                                      round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)),
                "traffic_ratio": (None if traffic is None else round(traffic / compulsory, 4)),
                "effective_gbs": round(effective, 1)}

    extra = {}
    if not args.no_extra:
        # FP64: the plain two-kernel path and the fused path, same workload and state
        p64 = Params(g=case["g"], theta=case["theta"], precision="f64", track_volume=True)
        d64 = device_inputs(mesh, case, p64)
        ws64 = mesh.workspace(p64, nsub)
        if prec != "f64":
            from paper_2311_08241_amd.autotune import autotune
            e64, u64 = d64["eta"].clone(), d64["U"].clone()

            def reset64():
                d64["eta"].copy_(e64)
                d64["U"].copy_(u64)
            t64 = autotune(mesh, lambda: step(d64, p64, ws64), "f64", nsub, top=24, log=log,
                           reset=reset64, use_cache=not args.retune)
            reset64()
            extra["fp64_plan"] = t64["plan"]
        for label, plain in (("fp64_plain", True), ("fp64_fused", False)):
            def s64():
                step(d64, p64, ws64, plain)
            s64()
            torch.cuda.synchronize()
            n = max(2, args.steps // 4)
            e0.record(stream)
            for _ in range(n):
                s64()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            extra[label] = {"value": float(mesh.nv) * nsub * n / (t * 1e-3),
                            "ms_per_step": t / n}
            log(f"[bench] {label}: {extra[label]['value']:.3e} vertex-substeps/s")
        extra["speedup_vs_fp64_plain"] = value / extra["fp64_plain"]["value"]
        del d64, ws64
        extra["sesm"] = bench_sesm(args, log, mesh, case, stream, not args.no_cpu)
        extra["trim_zstar"] = bench_trim(args, log, mesh, case, stream)
        extra["forcing"] = bench_forcing(args, log, mesh, case, stream)
        extra["visc"] = bench_visc(args, log, mesh, case, stream)
        if not args.small:
            extra["share_1_of_8"] = bench_share(args, log, mesh, case, value)

    cpu = None
    errors = None
    if not args.no_cpu:
        import oracle
        t0 = time.time()
        om = oracle.Mesh(case, reordered=True)
        log(f"[bench] oracle mesh {time.time() - t0:.1f}s")
        kw = dict(H0=om.v_in(case["H0"]), f=om.e_in(case["f"]), R=om.e_in(case["R"]),
                  g=case["g"], theta=case["theta"], nsub=nsub, tau=tau, linear_h=False,
                  volume=True)
        eta, U = om.v_in(case["eta0"]), om.e_in(case["U0"])
        # all cores: the ERR_STEPS chained steps of the error report, each timed
        t_all = []
        e_c, U_c = eta, U
        first = None
        for k in range(ERR_STEPS):
            t1 = time.perf_counter()
            e_c, U_c, ua_c, _ = om.subcycle(e_c, U_c, threads=0, **kw)
            t_all.append(time.perf_counter() - t1)
            if k == 0:
                first = (e_c, U_c, ua_c)
        cores = om.threads_used
        # one thread: the first step, three times
        t_one = []
        for _ in range(3):
            t1 = time.perf_counter()
            o1 = om.subcycle(eta, U, **kw)
            t_one.append(time.perf_counter() - t1)
        if not all(np.array_equal(a, b) for a, b in zip(o1[:3], first)):
            raise RuntimeError("threaded oracle differs from the serial oracle")
        per_step = om.nv * nsub
        med_all, med_one = float(np.median(t_all)), float(np.median(t_one))
        cpu = {"value": per_step / med_all, "unit": "vertex-substeps/s", "cores": cores,
               "kind": "oracle", "host_cpu": host_cpu(), "host_cpus": os.cpu_count(),
               "sample": f"median of {ERR_STEPS} chained baroclinic steps ({nsub} substeps "
                         f"each, {sum(t_all):.1f} s in all) of the same mesh, FP64, "
                         f"{cores} OpenMP threads (the multithreaded form, equal to the "
                         f"serial oracle bit for bit)",
               "single_thread": {"value": per_step / med_one, "cores": 1,
                                 "sample": f"median of 3 runs of the first baroclinic step, "
                                           f"{sum(t_one):.1f} s in all"},
               "speedup_all_cores": med_one / med_all}
        log(f"[bench] oracle: {cores} threads {med_all:.2f} s/step, 1 thread {med_one:.2f} "
            f"s/step ({cpu['value']:.3e} / {cpu['single_thread']['value']:.3e} "
            f"vertex-substeps/s)")
        # errors of the benchmarked configuration after ERR_STEPS steps
        eta_g = mesh.v_out(eta_err)
        eta_r = om.v_out(e_c)
        ua_g = mesh.e_out(Uavg_err)
        ua_r = om.e_out(ua_c)
        Av = om.v_out(om.Av)
        Ae = om.e_out(om.Ae)
        ref = case["eta_ref"] if prec == "f32" else 0.0
        den = np.abs(eta_r - ref).max()
        errors = {
            "after_substeps": nsub * ERR_STEPS, "plan": list(plan),
            "eta_max": float(np.abs(eta_g - eta_r).max() / den),
            "eta_rms": float(np.sqrt(np.sum(Av * (eta_g - eta_r) ** 2) /
                                     np.sum(Av * (eta_r - ref) ** 2))),
            "Uavg_max": float(np.abs(ua_g - ua_r).max() / np.abs(ua_r).max()),
            "Uavg_rms": float(np.sqrt(np.sum(Ae[:, None] * (ua_g - ua_r) ** 2) /
                                      np.sum(Ae[:, None] * ua_r ** 2))),
        }
        log(f"[bench] errors vs oracle: {errors}")

    if not args.no_extra:
        extra["batched"] = bench_batched(args, log, not args.no_cpu)
        extra["adjoint"] = bench_adjoint(args, log)

    out = {
        "metric": METRIC, "value": value, "unit": "vertex-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": f"{case['name']} lat-lon, 30% land, {nsub} substeps/step",
                   "nv": mesh.nv, "ne": mesh.ne, "substeps_per_step": nsub,
                   "precision": ("FP32 bulk, FP64 volume and averaged transport"
                                 if prec == "f32" else "FP64"),
                   "plan": {"tile": plan[0], "k_fused": plan[1], "block": plan[2]},
                   **({"variant": {"scheme": args.scheme, "visc": args.visc or None},
                       "note": "profiling run of another tile-kernel form; the roofline "
                               "bytes are those of the forward-backward scheme"}
                      if variant else {})},
        "roofline": roofline, "cpu_baseline": cpu, "errors": errors,
        "volume_drift": volume_drift, "hbm_gbs_algorithmic": round(achieved, 1),
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
