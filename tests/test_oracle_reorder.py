"""Pins of the oracle's space-filling-curve reordering.

The paper fixes nothing here; the pins are the defining properties of a
Hilbert curve (bijection onto 0..n^2-1, consecutive indices on edge-adjacent
cells, start at (0,0) and end at (n-1,0)), validity of the permutations and
CSR, and invariance of the physics under relabelling of the input.
"""
import numpy as np
import pytest

import oracle
import sesynth


@pytest.mark.parametrize("side", [2, 4, 16, 64])
def test_hilbert_is_a_hilbert_curve(side):
    d_of = {}
    for x in range(side):
        for y in range(side):
            d_of[(x, y)] = oracle.hilbert_d(side, x, y)
    assert sorted(d_of.values()) == list(range(side * side))
    cell = {d: xy for xy, d in d_of.items()}
    assert cell[0] == (0, 0) and cell[side * side - 1] == (side - 1, 0)
    for d in range(side * side - 1):
        (x0, y0), (x1, y1) = cell[d], cell[d + 1]
        assert abs(x0 - x1) + abs(y0 - y1) == 1


def test_hilbert_order2_table():
    """Order-2 curve visits the four quadrants (0,0) (0,1) (1,1) (1,0)."""
    seq = sorted(((oracle.hilbert_d(2, x, y), (x, y)) for x in range(2) for y in range(2)))
    assert [c for _, c in seq] == [(0, 0), (0, 1), (1, 1), (1, 0)]


@pytest.mark.parametrize("kind", ["jitter76", "chan54", "sphere86", "torus43"])
def test_reorder_is_valid(kind):
    mesh = sesynth.tiny_mesh(kind)
    vperm, eperm, tri_new, row_ptr, col = oracle.reorder(mesh)
    nv, ne = mesh["x"].size, mesh["tri"].shape[0]
    assert sorted(vperm) == list(range(nv)) and sorted(eperm) == list(range(ne))
    vinv = np.empty(nv, np.int64)
    vinv[vperm] = np.arange(nv)
    for e in range(ne):
        old = list(vinv[mesh["tri"][eperm[e]]])
        t = list(tri_new[e])
        assert t[0] == min(t)
        assert any(old[k:] + old[:k] == t for k in range(3))    # cyclic rotation, same orientation
    assert all(tuple(tri_new[e]) < tuple(tri_new[e + 1]) for e in range(ne - 1))
    assert row_ptr[0] == 0 and row_ptr[-1] == 3 * ne
    seen = set()
    for v in range(nv):
        es = [c >> 2 for c in col[row_ptr[v]:row_ptr[v + 1]]]
        assert es == sorted(es)
        for c in col[row_ptr[v]:row_ptr[v + 1]]:
            assert tri_new[c >> 2][c & 3] == v
            seen.add(int(c))
    assert len(seen) == 3 * ne


def test_reorder_keys_follow_curve():
    mesh = sesynth.planar_grid(16, 16, 1.0, 1.0)
    vperm, *_ = oracle.reorder(mesh)
    pts = np.column_stack([mesh["x"][vperm], mesh["y"][vperm]])
    steps = np.abs(np.diff(pts, axis=0)).sum(axis=1)
    assert np.all(steps == 1.0)     # the 16x16 lattice is visited along the curve


def test_duplicate_triangle_is_rejected():
    mesh = sesynth.tiny_mesh("two")
    mesh = dict(mesh)
    mesh["tri"] = np.array([[0, 1, 2], [0, 2, 3], [1, 2, 0]], np.int32)
    with pytest.raises(RuntimeError):
        oracle.reorder(mesh)


def test_physics_is_invariant_under_input_relabelling():
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=61)
    r = sesynth.rng(62)
    nv, ne = case["H0"].size, case["f"].size
    pv = r.permutation(nv)
    pe = r.permutation(ne)
    inv_v = np.empty(nv, np.int64)
    inv_v[pv] = np.arange(nv)
    rc = dict(case)
    rc["x"], rc["y"] = case["x"][pv], case["y"][pv]
    rc["tri"] = inv_v[case["tri"][pe]].astype(np.int32)
    rc["H0"], rc["eta0"] = case["H0"][pv], case["eta0"][pv]
    rc["f"], rc["R"], rc["U0"] = case["f"][pe], case["R"][pe], case["U0"][pe]
    a = oracle.run_case(case, nsteps=1)
    b = oracle.run_case(rc, nsteps=1)
    # canonical order makes the two runs identical, bit for bit
    assert np.array_equal(a["eta"], b["eta"]) and np.array_equal(a["Uavg"], b["Uavg"])
    assert np.array_equal(a["mesh"].tri, b["mesh"].tri)
