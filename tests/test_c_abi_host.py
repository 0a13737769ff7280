"""The C ABI from C: tests/c/abi_host.c includes include/sesub.h, links the built
library and makes host calls only (a host-only mesh, its reordering and geometry,
plan statistics, the AB3-AM4 coefficients, error statuses).  Its output is
compared with the oracle's independent reordering and geometry, with closed forms
and with the header's status codes.  No GPU, no Python between the caller and the
library."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2311_08241_amd")

N, H = 9, 1000.0


def _grid():
    """The program's mesh: N x N vertices of spacing H, cells split along the
    diagonal from the lower-left corner, counter-clockwise triangles."""
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x = (i * H).ravel().astype(np.float64)
    y = (j * H).ravel().astype(np.float64)
    tri = []
    for jj in range(N - 1):
        for ii in range(N - 1):
            a = jj * N + ii
            b, c, d = a + 1, a + N, a + N + 1
            tri += [[a, b, d], [a, d, c]]
    return dict(x=x, y=y, tri=np.array(tri, np.int32), periodic_x=False, periodic_y=False,
                period_x=0.0, period_y=0.0, spherical=False, radius=0.0)


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    if not os.path.exists(os.path.join(LIBDIR, "libsesub.so")):
        pytest.fail("libsesub.so is not built (python -c 'import __graft_entry__ as g; g.build()')")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path_factory.mktemp("cabi") / "abi_host")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_host.c"),
                    "-L", LIBDIR, "-lsesub", "-Wl,-rpath," + LIBDIR, "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    rows = {}
    for line in out.splitlines():
        k, *v = line.split()
        rows[k] = v
    assert "done" in rows
    return rows


def test_reordering_and_csr_from_c_equal_the_oracle(run):
    mesh = _grid()
    vperm, eperm, tri, row, col = oracle.reorder(mesh)
    nv, ne = N * N, 2 * (N - 1) ** 2
    assert [int(v) for v in run["info"][:3]] == [nv, ne, 3 * ne]
    assert np.array_equal(np.array(run["vperm"], np.int64), vperm)
    assert np.array_equal(np.array(run["eperm"], np.int64), eperm)
    assert np.array_equal(np.array(run["row_ptr"], np.int64), row)


def test_geometry_from_c_closes(run):
    sav, sae, gmax = (float(v) for v in run["areas"])
    area = ((N - 1) * H) ** 2
    assert sav == area and sae == area     # dual cells and triangles tile the square
    assert gmax == 0.0                     # grad N of a triangle sums to zero


def test_plan_stats_and_coefficients_from_c(run):
    ntiles, max_tri, max_vtx, ept, ok32, ok64 = (int(v) for v in run["plan"])
    assert ntiles == -(-N * N // 64) and ept == 1 and ok32 == 1 and ok64 == 1
    assert max_vtx <= N * N and max_tri <= 2 * (N - 1) ** 2
    beta, delta, gamma, zeta = (float(v) for v in run["sesm"])
    chi = 0.14 / 2      # eq. (eqdp_4) with theta = 0.14; eq. (eqdp_6), second line
    assert beta == 0.281105
    assert abs(zeta - (0.010 - 0.135 * chi)) <= 1e-16
    assert abs(gamma - (0.083 - 0.514 * chi)) <= 1e-16
    assert abs(delta - (2 * chi + gamma + 2 * zeta + 0.5)) <= 1e-15


def test_error_statuses_from_c(run):
    SE_ERR_ARG, SE_ERR_MESH = 1, 2
    assert run["err_null"] == [str(SE_ERR_ARG), "1"]          # with a message
    assert run["err_index"] == [str(SE_ERR_MESH), "1"]
    assert run["err_orientation"] == [str(SE_ERR_MESH), "1"]
    assert run["err_plan"] == [str(SE_ERR_ARG)]
    assert run["err_sesm"] == [str(SE_ERR_ARG)]
    assert run["err_host_only"] == [str(SE_ERR_ARG), "1"]   # no kernels on a host-only mesh
