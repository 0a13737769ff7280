"""Host-side checks of the GPU library that need no GPU.

The library is loaded and its exported symbols checked against the header;
meshes are created host-only (device -1), which runs the library's own
reordering and FP64 geometry, and compared integer for integer with the
oracle's independent implementation.  Argument and CFL errors are forced from
the host.
"""
import ctypes

import numpy as np
import pytest

import oracle
import sesynth
from oracle import brute
from paper_2311_08241_amd import _lib as L
from paper_2311_08241_amd import Mesh, Params


def test_library_exports_every_header_function():
    lib = L.lib()
    names = L.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def _cases():
    yield "jitter76", sesynth.tiny_mesh("jitter76")
    yield "chan54", sesynth.tiny_mesh("chan54")
    yield "sphere86", sesynth.tiny_mesh("sphere86")
    yield "torus43", sesynth.tiny_mesh("torus43")
    yield "C1", sesynth.basin_c1()
    yield "C2small", sesynth.channel_c2(nx=96, ny=40, nsteps=1)
    yield "C3small", sesynth.latlon_c3(nlon=128, nlat=96, nsteps=1)
    yield "C5small", sesynth.adjoint_c5(n=48)


@pytest.mark.parametrize("name,mesh", list(_cases()))
def test_reorder_and_geometry_match_oracle_exactly(name, mesh):
    m = Mesh.from_dict(mesh, device=-1)
    vperm, eperm, tri, row, col = oracle.reorder(mesh)
    assert np.array_equal(m.vperm, vperm) and np.array_equal(m.eperm, eperm)
    t2, r2, c2 = m.csr()
    assert np.array_equal(t2, tri) and np.array_equal(r2, row) and np.array_equal(c2, col)
    Av, Ae, gN = m.geometry()
    om = oracle.Mesh(mesh, reordered=True)
    assert np.array_equal(Av, om.Av) and np.array_equal(Ae, om.Ae) and np.array_equal(gN, om.gN)


def _full_size():
    yield "C2", lambda: sesynth.channel_c2(nsteps=1)
    yield "C3", lambda: sesynth.latlon_c3(nsteps=1)
    yield "C5", lambda: sesynth.adjoint_c5()


@pytest.mark.parametrize("name,make", list(_full_size()), ids=[c[0] for c in _full_size()])
def test_full_size_reorder_and_geometry_match_oracle_exactly(name, make):
    """The workloads at their full sizes (0.5M, 2.2M and 65k vertices): permutations,
    canonical triangles, CSR, A_v, A_e and grad N integer for integer and bit for bit."""
    mesh = make()
    m = Mesh.from_dict(mesh, device=-1)
    om = oracle.Mesh(mesh, reordered=True)
    assert np.array_equal(m.vperm, om.vperm) and np.array_equal(m.eperm, om.eperm)
    t2, r2, c2 = m.csr()
    assert np.array_equal(t2, om.tri) and np.array_equal(r2, om.row_ptr)
    assert np.array_equal(c2, om.col)
    Av, Ae, gN = m.geometry()
    assert np.array_equal(Av, om.Av) and np.array_equal(Ae, om.Ae) and np.array_equal(gN, om.gN)


def test_sesm_coefficients_match_the_oracle_settings():
    """se_sesm_coefficients against the oracle's own reading of eqs. (eqdp_4), (eqdp_6)."""
    from oracle import analytic
    from paper_2311_08241_amd.api import sesm_coefficients
    for theta in (0.0, 0.14, 0.3):
        assert np.allclose(sesm_coefficients(theta), analytic.sesm_params(theta), rtol=0,
                           atol=1e-15)
    assert sesm_coefficients(0.14, 0.2)[0] == 0.2
    with pytest.raises(L.SeError):
        sesm_coefficients(float("nan"))


@pytest.mark.parametrize("name,mesh", list(_cases())[:6])
def test_viscous_neighbours_and_edge_geometry_match_oracle_exactly(name, mesh):
    """The library finds neighbours through its CSR rows, the oracle by sorting
    vertex pairs; the edge geometry is the same written definition in both."""
    m = Mesh.from_dict(mesh, device=-1)
    nb, ln, lod = m.neighbours()
    om = oracle.Mesh(mesh, reordered=True)
    nb2, ln2, lod2 = om.visc_geometry()
    assert np.array_equal(nb, nb2)
    assert np.array_equal(ln, ln2) and np.array_equal(lod, lod2)


@pytest.mark.parametrize("kind", ["jitter65", "chan54", "torus43", "grid3"])
def test_mu_max_bounds_the_spectrum(kind):
    mesh = sesynth.tiny_mesh(kind)
    m = Mesh.from_dict(mesh, device=-1)
    ops = brute.dense_operators(mesh)
    mu = np.linalg.eigvals(-ops["D"] @ ops["G"]).real.max()
    assert m.mu_max >= mu * (1 - 1e-12)
    assert m.mu_max <= 3.0 * mu


def test_mu_max_is_tight_on_a_split_torus():
    t = sesynth.torus(8, 6, 1000.0, 1300.0)
    m = Mesh.from_dict(t, device=-1)
    expect = 4 / 1000.0 ** 2 + 4 / 1300.0 ** 2     # 5-point Laplacian at the Nyquist mode
    assert abs(m.mu_max - expect) <= 1e-12 * expect


def _desc(x, y, tri, flags=0, px=0.0, py=0.0, radius=0.0):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    d = L.MeshDesc(x.size, tri.shape[0], x.ctypes.data_as(ctypes.c_void_p),
                   y.ctypes.data_as(ctypes.c_void_p), tri.ctypes.data_as(ctypes.c_void_p),
                   flags, px, py, radius)
    return d, (x, y, tri)


def _create(d):
    h = ctypes.c_void_p()
    st = L.lib().se_mesh_create(ctypes.byref(d), -1, ctypes.byref(h))
    if st == 0:
        L.lib().se_mesh_destroy(h)
    return st


def test_mesh_errors():
    x = [0.0, 1.0, 1.0, 0.0]
    y = [0.0, 0.0, 1.0, 1.0]
    assert _create(_desc(x, y, [[0, 1, 2], [0, 2, 3]])[0]) == L.SE_OK
    assert _create(_desc(x, y, [[0, 1, 2], [0, 2, 4]])[0]) == L.SE_ERR_MESH      # index range
    assert _create(_desc(x, y, [[0, 2, 1], [0, 2, 3]])[0]) == L.SE_ERR_MESH      # clockwise
    assert _create(_desc(x, y, [[0, 1, 2], [1, 2, 0]])[0]) == L.SE_ERR_MESH      # duplicate
    assert _create(_desc(x, y, [[0, 1, 1], [0, 2, 3]])[0]) == L.SE_ERR_MESH      # repeated vertex
    assert _create(_desc(x + [5.0], y + [5.0], [[0, 1, 2], [0, 2, 3]])[0]) == L.SE_ERR_MESH  # orphan
    assert _create(_desc(x, y, np.zeros((0, 3)))[0]) == L.SE_ERR_ARG
    assert _create(_desc(x, y, [[0, 1, 2], [0, 2, 3]], flags=L.SE_SPHERICAL)[0]) == L.SE_ERR_ARG
    assert _create(_desc([0.0, 1.0, np.nan, 0.0], y, [[0, 1, 2], [0, 2, 3]])[0]) == L.SE_ERR_MESH


def _call_subcycle(mesh, params, nsub=10, dt=100.0, null_eta=False):
    dummy = ctypes.c_void_p(256)
    st = L.State(None if null_eta else dummy, dummy, None, None)
    fo = L.Forcing(dummy, dummy, dummy, None)
    pc = params.c()
    return L.lib().se_subcycle(mesh.handle, ctypes.byref(pc), ctypes.byref(st), ctypes.byref(fo),
                               nsub, dt, dummy, None)


def test_subcycle_argument_and_cfl_errors():
    mesh = sesynth.tiny_mesh("jitter65")
    m = Mesh.from_dict(mesh, device=-1)
    ok = Params(h_max=100.0, check_cfl=True)
    # within the bound: fails only because the mesh is host-only
    assert _call_subcycle(m, ok, nsub=10, dt=10.0) == L.SE_ERR_ARG
    lim = 2 / np.sqrt(1 + 2 * 0.14)
    dts_lim = lim / np.sqrt(9.81 * 5000.0 * m.mu_max)
    hot = Params(h_max=5000.0, check_cfl=True)
    assert _call_subcycle(m, hot, nsub=10, dt=10 * dts_lim * 1.01) == L.SE_ERR_CFL
    assert _call_subcycle(m, hot, nsub=10, dt=10 * dts_lim * 0.99) == L.SE_ERR_ARG
    assert _call_subcycle(m, Params(h_max=0.0, check_cfl=True)) == L.SE_ERR_ARG
    assert _call_subcycle(m, Params(), nsub=0) == L.SE_ERR_ARG
    assert _call_subcycle(m, Params(), dt=-1.0) == L.SE_ERR_ARG
    assert _call_subcycle(m, Params(), dt=float("nan")) == L.SE_ERR_ARG
    assert _call_subcycle(m, Params(g=0.0)) == L.SE_ERR_ARG
    assert _call_subcycle(m, Params(), null_eta=True) == L.SE_ERR_ARG
    bad = Params()
    pc = bad.c()
    pc.precision = 7
    dummy = ctypes.c_void_p(256)
    st = L.State(dummy, dummy, None, None)
    fo = L.Forcing(dummy, dummy, dummy, None)
    assert L.lib().se_subcycle(m.handle, ctypes.byref(pc), ctypes.byref(st), ctypes.byref(fo),
                               5, 1.0, dummy, None) == L.SE_ERR_ARG
    assert b"precision" in L.lib().se_last_error()


def test_workspace_size_grows_with_substeps():
    m = Mesh.from_dict(sesynth.tiny_mesh("jitter76"), device=-1)
    a = m.workspace_bytes(Params(), 10)
    b = m.workspace_bytes(Params(), 100)
    c = m.workspace_bytes(Params(precision="f32"), 10)
    assert b > a > c > 0 and a % 256 == 0


def test_plan_halves_the_few_tiles_above_the_next_lower_tier():
    """Tiles of T consecutive vertices, except that when at most one tile in 50 holds more
    local triangles than the register tier below the one the largest tile needs, those
    tiles are halved (here: one of 71 at 464,4,512, four of 256 at 128,4,256 on the
    256 x 128 channel), so the plan keeps the smaller tier; where more tiles exceed it the
    tiles stay uniform."""
    case = sesynth.channel_c2(nx=256, ny=128, nsteps=1)
    mesh = Mesh.from_dict(case, device=-1)
    nv = mesh.nv
    for plan, ntiles, tier in (((464, 4, 512), 72, 4), ((128, 4, 256), 260, 3)):
        st = mesh.plan_stats(*plan)
        assert st["ntiles"] == ntiles > -(-nv // plan[0])
        assert st["tri_per_thread"] == tier and st["max_tri"] <= tier * plan[2]
    st = mesh.plan_stats(576, 4, 512)      # many tiles above 3 x 512: uniform
    assert st["ntiles"] == -(-nv // 576)


def test_autotune_candidates_and_signature_on_a_host_mesh():
    """The tuner's host side: plan ranking for both schemes and the cache key."""
    from paper_2311_08241_amd import Mesh
    from paper_2311_08241_amd import autotune as A
    case = sesynth.channel_c2(nx=64, ny=48, nsteps=1)
    m = Mesh.from_dict(case, device=-1)
    for prec in ("f32", "f64", "f32-sesm", "f64-sesm"):
        c = A.candidates(m, prec, case["nsub"], top=8)
        assert c and all(len(r) == 5 for r in c)
        assert [r[0] for r in c] == sorted(r[0] for r in c)
        lkey = "lds_" + ("sesm_" if prec.endswith("sesm") else "") + prec[:3]
        assert all(r[4][lkey] <= A.LDS_MAX for r in c)
    # viscous form: two rings per substep (k_fused even, >= 2), its register tiers and
    # the velocity array in LDS
    for prec in ("f32-visc", "f64-visc"):
        c = A.candidates(m, prec, case["nsub"], top=8)
        assert c and all(r[2] >= 2 and r[2] % 2 == 0 for r in c)
        es = 4 if prec.startswith("f32") else 8
        assert all(r[4]["lds_" + prec[:3]] + 2 * es * r[4]["max_tri"] <= A.LDS_MAX for r in c)
    assert not A._tier_ok("f32-visc", 4, 1024) and A._tier_ok("f32-visc", 3, 1024)
    sig = A.mesh_signature(m)
    assert isinstance(sig, str) and len(sig) == 20 and sig == A.mesh_signature(m)
    with pytest.raises(ValueError):
        A._split("f16")
