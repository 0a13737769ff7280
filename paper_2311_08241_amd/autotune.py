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

TILES = (128, 256, 384, 512, 768, 1024)
KS = (1, 2, 3, 4, 5, 6, 8)
BLOCKS = (256, 512)
CACHE = os.environ.get("SESUB_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "sesub_plans.json"))


def mesh_signature(mesh) -> str:
    if hasattr(mesh, "signature"):
        return hashlib.sha256(mesh.signature().encode()).hexdigest()[:20]
    h = hashlib.sha256()
    tri, row, col = mesh.csr()
    h.update(np.int64([mesh.nv, mesh.ne]).tobytes())
    h.update(tri.tobytes())
    return h.hexdigest()[:20]


def candidates(mesh, precision: str, nsub: int, top: int = 8):
    """Feasible plans ranked by modelled bytes per vertex-substep."""
    key = "ok_f32" if precision == "f32" else "ok_f64"
    bkey = "bytes_per_vs_f32" if precision == "f32" else "bytes_per_vs_f64"
    out = []
    # at fixed (K, B) a larger tile has less halo and less modelled traffic, so only
    # the largest feasible tile and the next smaller one are kept
    for K in KS:
        if K > nsub:
            continue
        for B in BLOCKS:
            kept = 0
            for T in sorted(TILES, reverse=True):
                try:
                    st = mesh.plan_stats(T, K, B)
                except Exception:
                    continue
                if not st[key]:
                    continue
                # a launch sequence with a short last chunk wastes part of a launch
                waste = (-(-nsub // K) * K) / nsub
                out.append((st[bkey] * waste, T, K, B, st))
                kept += 1
                if kept == 2:
                    break
    out.sort(key=lambda r: r[0])
    return out[:top]


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


def autotune(mesh, run_step, precision: str, nsub: int, *, top: int = 8, reps: int = 3,
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
        table.append({"plan": [T, K, B], "ms": ms, "model_bytes_per_vs": model,
                      "tri_overhead": st["tri_overhead"]})
        if log:
            log(f"[tune] T={T} K={K} B={B}: {ms:.3f} ms/step (model {model:.1f} B/vs, "
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
