"""Plan autotuner for the temporally blocked subcycle kernel.

Candidates (vertices per tile, substeps per launch, workgroup size) are
filtered on the host by se_plan_stats (register and LDS budget of the
requested precision) and ranked by the modelled device-memory bytes per
vertex-substep; the best-ranked few are timed on the GPU with the caller's
state and the fastest is installed with se_set_plan.  Results are cached per
(device name, precision, mesh signature, substep count) in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

TILES = (256, 384, 512, 768, 1024)
KS = (2, 3, 4, 5, 6, 8)
BLOCKS = (256, 512, 1024)
EPT_TIERS = (1, 2, 3, 4, 6, 8)
LDS_MAX = 160 * 1024
CACHE = os.environ.get("SESUB_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "sesub_plans.json"))


def _tier_ok(precision: str, ept: int, block: int) -> bool:
    """Register tiers the library runs without spills (mirror of its plan check)."""
    if block == 256:
        return ept <= (8 if precision == "f32" else 6)
    if block == 512:
        return ept <= (8 if precision == "f32" else 4)
    return ept <= (4 if precision == "f32" else 1)


def mesh_signature(mesh) -> str:
    if hasattr(mesh, "signature"):
        return hashlib.sha256(mesh.signature().encode()).hexdigest()[:20]
    h = hashlib.sha256()
    tri, row, col = mesh.csr()
    h.update(np.int64([mesh.nv, mesh.ne]).tobytes())
    h.update(tri.tobytes())
    return h.hexdigest()[:20]


def candidates(mesh, precision: str, nsub: int, top: int = 18):
    """Feasible plans: a diverse shortlist ranked by modelled traffic and halo work.

    One se_plan_stats call per (tile, k) gives the largest triangle count of a tile;
    the register tier of each workgroup size follows from it.  From every
    (workgroup size, tier) group the three best-scoring plans are kept, so that
    plans of different occupancy are all timed.
    """
    lkey = "lds_f32" if precision == "f32" else "lds_f64"
    bkey = "bytes_per_vs_f32" if precision == "f32" else "bytes_per_vs_f64"
    b_stream = 236.0 if precision == "f32" else 356.0   # one streaming pass per substep
    groups = {}
    for K in KS:
        if K > nsub:
            continue
        for T in TILES:
            try:
                st = mesh.plan_stats(T, K, 256)
            except Exception:
                continue
            if st[lkey] > LDS_MAX:
                continue
            waste = (-(-nsub // K) * K) / nsub     # short last chunk of the launch sequence
            for B in BLOCKS:
                need = -(-st["max_tri"] // B)
                ept = next((e for e in EPT_TIERS if e >= need), None)
                if ept is None or not _tier_ok(precision, ept, B):
                    continue
                # relative device traffic plus relative triangle work (the halo rings
                # are recomputed; on average half of the outermost ring's overhead)
                score = (st[bkey] / b_stream + 0.5 * (1.0 + st["tri_overhead"])) * waste
                groups.setdefault((B, ept), []).append((score, T, K, B, st))
    short = []
    for g in groups.values():
        g.sort(key=lambda r: r[0])
        short.extend(g[:4])
    short.sort(key=lambda r: r[0])
    return short[:top]


def _load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except Exception:
        return {}


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def autotune(mesh, run_step, precision: str, nsub: int, *, top: int = 18, reps: int = 3,
             use_cache: bool = True, log=None, reset=None):
    """Pick and install the fastest plan.

    run_step() must perform one se_subcycle call with the mesh's current plan
    on the caller's stream; reset(), if given, restores the state before each
    candidate (outside the timed region) so long tuning runs stay physical.
    Returns dict(plan=(T, K, B), ms=..., table=[...]).
    """
    import torch
    props = torch.cuda.get_device_properties(mesh.device)
    dev = f"{getattr(props, 'gcnArchName', '?')}x{props.multi_processor_count}"
    key = f"{dev}|{precision}|{mesh_signature(mesh)}|{nsub}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        T, K, B = cache[key]["plan"]
        mesh.set_plan(T, K, B)
        return dict(cache[key], cached=True)
    table = []
    best = None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for model, T, K, B, st in candidates(mesh, precision, nsub, top):
        t0 = time.time()
        mesh.set_plan(T, K, B)
        if reset is not None:
            reset()
        run_step()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            run_step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        table.append({"plan": [T, K, B], "ms": ms, "score": model,
                      "tri_overhead": st["tri_overhead"]})
        if log:
            log(f"[tune] T={T} K={K} B={B}: {ms:.3f} ms/step (score {model:.2f}, "
                f"setup {time.time() - t0:.1f}s)")
        if best is None or ms < best[0]:
            best = (ms, T, K, B)
    if best is None:
        raise RuntimeError("autotune: no feasible plan")
    mesh.set_plan(*best[1:])
    res = {"plan": list(best[1:]), "ms": best[0], "table": table}
    if use_cache:
        cache = _load_cache()
        cache[key] = res
        _save_cache(cache)
    return dict(res, cached=False)
