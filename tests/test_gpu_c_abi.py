"""The C ABI from a plain C program on the GPU: tests/c/abi_gpu (built by
__graft_entry__.build()) creates the mesh (planar, periodic or spherical),
allocates device memory with hipMalloc,
runs one FP64 se_subcycle with the volume tracked and copies the results back, with
no Python or torch between it and the library.  Its eta, U, <<U>> and volume series
equal the oracle's within 1e-12 (Sec. 2.2, eqs. (eq4_10) and (eq4_12))."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import sesynth

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "abi_gpu")


def _write_input(path, c):
    from paper_2311_08241_amd import _lib as L
    nv, ne = c["x"].size, c["tri"].shape[0]
    mflags = ((L.SE_PERIODIC_X if c["periodic_x"] else 0) | (L.SE_PERIODIC_Y if c["periodic_y"] else 0)
              | (L.SE_SPHERICAL if c["spherical"] else 0))
    pflags = 1 if c["linear_h"] else 0    # SE_LINEAR_H
    with open(path, "wb") as f:
        np.array([nv, ne], np.int64).tofile(f)
        np.array([c["nsub"], mflags, pflags, 0], np.int32).tofile(f)
        np.array([c["tau"], c["g"], c["theta"], c["period_x"], c["period_y"], c["radius"]],
                 np.float64).tofile(f)
        for a in (c["x"], c["y"]):
            np.ascontiguousarray(a, np.float64).tofile(f)
        np.ascontiguousarray(c["tri"], np.int32).tofile(f)
        for a in (c["eta0"], c["U0"], c["R"], c["f"], c["H0"]):
            np.ascontiguousarray(a, np.float64).tofile(f)


@pytest.mark.parametrize("name", ["jitter", "channel", "sphere"])
def test_c_caller_fp64_subcycle_equals_oracle(tmp_path, name):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (python -c 'import __graft_entry__ as g; g.build()')")
    if name == "jitter":
        c = sesynth.random_case(sesynth.planar_grid(61, 47, 1300.0, 1100.0, jitter=0.3,
                                                    r=sesynth.rng(21)), seed=9, nsub=17)
        c["tau"] = 17 * 3.0
    elif name == "channel":   # periodic in x
        c = sesynth.channel_c2(nx=96, ny=40, nsteps=1)
    else:                     # longitude and latitude on the sphere
        c = sesynth.latlon_c3(nlon=96, nlat=64, nsteps=1)
        c["tau"] = c["nsub"] * 200.0
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    _write_input(inp, c)
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    nv, ne, ns = c["x"].size, c["tri"].shape[0], c["nsub"]
    o = np.fromfile(out, np.float64)
    assert o.size == nv + 4 * ne + ns + 1
    eta, U, Ua, vol = (o[:nv], o[nv:nv + 2 * ne].reshape(ne, 2),
                       o[nv + 2 * ne:nv + 4 * ne].reshape(ne, 2), o[nv + 4 * ne:])
    m = oracle.Mesh(c, reordered=True)
    ref = oracle.run_case(c, nsteps=1, mesh=m)
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(eta, m.v_out(ref["eta"])) <= 1e-12
    assert rel(U, m.e_out(ref["U"])) <= 1e-12
    assert rel(Ua, m.e_out(ref["Uavg"])) <= 1e-12
    assert np.abs(vol - ref["volume"]).max() <= 1e-12 * np.abs(ref["volume"]).max()
