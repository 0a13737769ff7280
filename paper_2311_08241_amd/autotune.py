"""Plan autotuner for the temporally blocked subcycle kernel.

Candidates (vertices per tile, substeps per launch, workgroup size) are
filtered on the host by se_plan_stats (register and LDS budget of the
requested precision) and ranked by a latency/occupancy model of one tile; the
best-ranked are timed on the GPU with the caller's state, the fastest few timed
again, and the winner is installed with se_set_plan.  Results are cached per
(device name, precision, mesh signature, substep count) in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

TILES = (256, 288, 304, 320, 336, 352, 384, 416, 448, 464, 480, 496, 512, 520, 576, 640, 768,
         1024)
KS = (2, 3, 4, 5, 6)
VISC_KS = (2, 4, 6, 8)
BLOCKS = (256, 512, 1024)
EPT_TIERS = (1, 2, 3, 4, 6, 8)
LDS_MAX = 160 * 1024
CACHE = os.environ.get("SESUB_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "sesub_plans.json"))
# plans tuned on MI355X for the synthetic workloads, consulted when CACHE has no
# entry (read-only; keys as in CACHE)
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_plans.json")


def _split(precision: str):
    """'f32' / 'f64', optionally with '-sesm' (the AB3-AM4 scheme) or '-visc' (the
    forward-backward scheme with the barotropic viscous term)."""
    prec, _, scheme = precision.partition("-")
    if prec not in ("f32", "f64") or scheme not in ("", "sesm", "visc"):
        raise ValueError(f"precision {precision!r}: expected f32 or f64, optionally with "
                         "-sesm or -visc")
    return prec, scheme == "sesm"


def _visc(precision: str) -> bool:
    return precision.endswith("-visc")


def _tier_ok(precision: str, ept: int, block: int) -> bool:
    """Register tiers the library runs without spills (mirror of its plan check)."""
    prec, sm = _split(precision)
    if _visc(precision):   # the library's viscous-form check
        if block == 1024:
            return ept <= (3 if prec == "f32" else 1)
        return ept <= (6 if prec == "f32" else 4) if block == 512 else True
    if block == 256:
        return ept <= (8 if prec == "f32" else 6)
    if block == 512:
        return ept <= (8 if prec == "f32" else 4)
    return ept <= ((3 if sm else 4) if prec == "f32" else (1 if sm else 3))


# VGPRs of the FP64 tile kernel per register tier, from the compiler's resource report
# (the per-triangle indices and geometry are re-materialised every substep)
_F64_VGPRS = {1: 82, 2: 101, 3: 127, 4: 157, 6: 215, 8: 256}
# the same for the viscous form (FP32 up to three slots: the edge geometry held in
# registers; the tiers the library refuses are never timed)
_VISC_VGPRS = {"f32": {1: 72, 2: 102, 3: 127, 4: 141, 6: 189, 8: 239},
               "f64": {1: 109, 2: 141, 3: 165, 4: 197, 6: 256, 8: 256}}


def _vgprs(precision: str, ept: int) -> int:
    """Approximate VGPRs of the tile kernel per register tier (measured from the
    compiler's resource report: about 24 per triangle slot in FP32, 26 with the two
    extra transports of the AB3-AM4 scheme, 51 in FP64 AB3-AM4; FP64 forward-backward
    and viscous tiers tabulated)."""
    prec, sm = _split(precision)
    if _visc(precision):
        v = _VISC_VGPRS[prec][ept]
    elif prec == "f32":
        v = 37 + 26 * ept if sm else 32 + 24 * ept
    else:
        v = 52 + 51 * ept if sm else _F64_VGPRS[ept]
    return -(-v // 8) * 8


def mesh_signature(mesh) -> str:
    if hasattr(mesh, "signature"):
        return hashlib.sha256(mesh.signature().encode()).hexdigest()[:20]
    h = hashlib.sha256()
    tri, row, col = mesh.csr()
    h.update(np.int64([mesh.nv, mesh.ne]).tobytes())
    h.update(tri.tobytes())
    return h.hexdigest()[:20]


def candidates(mesh, precision: str, nsub: int, top: int = 30):
    """Feasible plans, ranked by a latency/occupancy model of one tile.

    A tile costs a fixed load/write-back latency plus, per substep, time
    proportional to its triangles per thread; tiles resident per CU follow from
    the register tier (VGPRs per wave) and the LDS size.  The estimate
    (tile time) / (vertex-substeps per tile x resident tiles) orders the plans;
    the shortlist is then timed.  One se_plan_stats call per (tile, k, block) gives
    the largest triangle count and the LDS size.
    """
    prec, sm = _split(precision)
    visc = _visc(precision)
    lkey = ("lds_sesm_" if sm else "lds_") + prec
    es = 4 if prec == "f32" else 8
    lat_us, sub_us = 5.8, 0.45      # load + write-back; per substep and triangle/thread
    rows = []
    for K in (VISC_KS if visc else KS):
        ks = K // 2 if visc else K     # substeps per launch (two rings each with the term)
        if ks > nsub:
            continue
        waste = (-(-nsub // ks) * ks) / nsub     # short last chunk of the launch sequence
        for T in TILES:
            for B in BLOCKS:
                # per block size: the plan halves its few oversized tiles against the
                # register tiers of that block size
                try:
                    st = mesh.plan_stats(T, K, B)
                except Exception:
                    continue
                lds = st[lkey] + (2 * es * st["max_tri"] if visc else 0)
                if lds > LDS_MAX:
                    continue
                need = -(-st["max_tri"] // B)
                ept = next((e for e in EPT_TIERS if e >= need), None)
                if ept is None or not _tier_ok(precision, ept, B):
                    continue
                waves = min(8, 512 // _vgprs(precision, ept))
                resident = min((4 * waves) // (B // 64), LDS_MAX // max(1, lds))
                if resident < 1:
                    continue
                tile_us = lat_us + ks * (1.5 if visc else 1.0) * sub_us * st["max_tri"] / B
                score = tile_us / (T * ks * resident) * waste * 1e3
                rows.append((score, T, K, B, st))
    rows.sort(key=lambda r: r[0])
    return rows[:top]


def _load_json(path):
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return {}


def _load_cache():
    return _load_json(CACHE)


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def autotune(mesh, run_step, precision: str, nsub: int, *, top: int = 30, reps: int = 3,
             final: int = 3, final_reps: int = 10, use_cache: bool = True, log=None,
             reset=None):
    """Pick and install the fastest plan.

    Every candidate is timed over `reps` steps; the `final` fastest are timed again
    over `final_reps` steps and the fastest of those is installed.
    run_step() must perform one se_subcycle call with the mesh's current plan
    on the caller's stream; reset(), if given, restores the state before each
    candidate (outside the timed region) so long tuning runs stay physical.
    Returns dict(plan=(T, K, B), ms=..., table=[...]).
    """
    import torch
    props = torch.cuda.get_device_properties(mesh.device)
    dev = f"{getattr(props, 'gcnArchName', '?')}x{props.multi_processor_count}"
    key = f"{dev}|{precision}|{mesh_signature(mesh)}|{nsub}"
    if use_cache:
        for src in (_load_cache(), _load_json(SHIPPED)):
            if key in src:
                T, K, B = src[key]["plan"]
                mesh.set_plan(T, K, B)
                return dict(src[key], cached=True)
    table = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(T, K, B, n):
        mesh.set_plan(T, K, B)
        if reset is not None:
            reset()
        run_step()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            run_step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    from ._lib import SeError
    for model, T, K, B, st in candidates(mesh, precision, nsub, top):
        t0 = time.time()
        try:
            ms = timed(T, K, B, reps)
        except SeError as err:   # outside the library's own budget check: skip
            if log:
                log(f"[tune] T={T} K={K} B={B}: skipped ({err})")
            continue
        table.append({"plan": [T, K, B], "ms": ms, "score": model,
                      "tri_overhead": st["tri_overhead"]})
        if log:
            log(f"[tune] T={T} K={K} B={B}: {ms:.3f} ms/step (score {model:.2f}, "
                f"setup {time.time() - t0:.1f}s)")
    if not table:
        raise RuntimeError("autotune: no feasible plan")
    best = None
    for row in sorted(table, key=lambda r: r["ms"])[:final]:
        ms = timed(*row["plan"], final_reps)
        row["ms_final"] = ms
        if log:
            log(f"[tune] final T={row['plan'][0]} K={row['plan'][1]} B={row['plan'][2]}: "
                f"{ms:.3f} ms/step")
        if best is None or ms < best[0]:
            best = (ms, *row["plan"])
    mesh.set_plan(*best[1:])
    res = {"plan": list(best[1:]), "ms": best[0], "table": table}
    if use_cache:
        cache = _load_cache()
        cache[key] = res
        _save_cache(cache)
    return dict(res, cached=False)
