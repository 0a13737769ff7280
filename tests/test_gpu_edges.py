"""Degenerate and ragged cases of the forward subcycle on the GPU, against the oracle.

* the smallest mesh, two triangles on four vertices (every vertex on the coast, one
  tile holding the whole mesh), with one substep and with a number of substeps that
  is not a multiple of the substeps per launch;
* one substep with a plan that fuses four (a single launch that stops after its first
  inner substep) and K n + 1 substeps (a last launch of one substep) on a mesh of
  many tiles;
* a tile size larger than the mesh.
FP64 within 1e-12 of the oracle (eta, U, <<U>>, volume); FP32 bit for bit equal to the
plain FP32 path, which itself stays within its rounding budget of the oracle.
"""
import numpy as np
import pytest

import sesynth
from test_gpu_forward import _lib_mesh, _params, _rel, _run_gpu, _run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _two(nsub):
    c = sesynth.random_case(sesynth.tiny_mesh("two"), seed=11, nsub=nsub)
    c["tau"] = 3.0 * nsub   # substeps of 3 s: within the CFL bound on 1 km cells
    return c


def _check_fp64(case, plans, nsteps=2):
    mesh = _lib_mesh(case)
    ref = _run_oracle(case, nsteps)
    for plan in plans:
        got = _run_gpu(case, mesh, _params(case), nsteps, plan=None if plan == "plain" else plan,
                       plain=plan == "plain")
        for g, e in zip(got[:3], ref[:3]):
            assert _rel(g, e) <= 1e-12, plan
        assert np.abs(got[3] - ref[3]).max() <= 1e-12 * max(np.abs(ref[3]).max(), 1e-300), plan
    return mesh


@pytest.mark.parametrize("nsub", [1, 2, 7])
def test_two_triangles(nsub):
    case = _two(nsub)
    mesh = _check_fp64(case, ["plain", (64, 1, 256), (64, 4, 256), (64, 8, 512)])
    p = _params(case, "f32")
    ref = _run_gpu(case, mesh, p, 2, plain=True)
    for plan in ((64, 1, 256), (64, 4, 256)):
        out = _run_gpu(case, mesh, p, 2, plan=plan)
        for a, b in zip(out[:3], ref[:3]):
            assert np.array_equal(a, b), plan


@pytest.mark.parametrize("nsub", [1, 9])
def test_ragged_substep_counts_on_many_tiles(nsub):
    case = sesynth.random_case(sesynth.planar_grid(45, 37, 1200.0, 1000.0, jitter=0.3,
                                                   r=sesynth.rng(78)), seed=5, nsub=nsub)
    case["tau"] = 2.5 * nsub   # within the CFL bound of the finest jittered cells
    _check_fp64(case, [(128, 4, 256), (256, 4, 512), (512, 4, 1024)], nsteps=3)


def test_tile_larger_than_the_mesh():
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=6, nsub=6)
    mesh = _lib_mesh(case)
    assert mesh.plan_stats(1024, 3, 512)["ntiles"] == 1
    _check_fp64(case, [(1024, 3, 512)])
