"""The multithreaded form of the oracle subcycle (the all-core CPU baseline of the
benchmark) against the plain serial definition.

The threaded form gathers each vertex's sub-cell fluxes in ascending triangle
order, the order in which the serial triangle loop adds them, so the elevation,
transport and averaged transport must be equal bit for bit for any thread count;
the volume is summed in fixed vertex blocks and must agree to rounding.
"""
import numpy as np
import pytest

import oracle
import sesynth


def _inputs(case, m, with_w):
    W = None
    if with_w:
        W = m.v_in(1e-6 * sesynth.rng(9).standard_normal(case["x"].size))
    return dict(H0=m.v_in(case["H0"]), f=m.e_in(case["f"]), R=m.e_in(case["R"]), W=W,
                g=case["g"], theta=case["theta"], nsub=case["nsub"], tau=case["tau"],
                linear_h=case["linear_h"])


CASES = [
    ("jitter76", lambda: sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=4, nsub=17)),
    ("chan54", lambda: sesynth.random_case(sesynth.tiny_mesh("chan54"), seed=5, nsub=11)),
    ("sphere86", lambda: sesynth.random_case(sesynth.tiny_mesh("sphere86"), seed=6, nsub=9)),
    ("grid 120x70", lambda: sesynth.random_case(
        sesynth.planar_grid(120, 70, 3000.0, 2800.0, jitter=0.3, r=sesynth.rng(3)), seed=7,
        nsub=12)),
    ("basin", lambda: sesynth.basin_c1()),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("with_w", [False, True])
def test_threaded_subcycle_equals_serial(name, make, with_w):
    case = make()
    m = oracle.Mesh(case, reordered=True)
    kw = _inputs(case, m, with_w)
    eta0, U0 = m.v_in(case["eta0"]), m.e_in(case["U0"])
    ref = m.subcycle(eta0, U0, **kw)
    for nt in (1, 3, 8):
        out = m.subcycle(eta0, U0, threads=nt, **kw)
        assert m.threads_used == nt
        for a, b in zip(out[:3], ref[:3]):
            assert np.array_equal(a, b), (name, nt)
        scale = np.sum(np.abs(m.Av * eta0)) + np.sum(np.abs(m.Av * out[0]))
        assert np.all(np.abs(out[3] - ref[3]) <= 1e-14 * scale)


def test_threaded_chained_steps_equal_serial():
    case = sesynth.random_case(sesynth.planar_grid(90, 60, 2500.0, 2500.0, jitter=0.3,
                                                   r=sesynth.rng(8)), seed=8, nsub=10)
    m = oracle.Mesh(case, reordered=True)
    kw = _inputs(case, m, False)
    e1, u1 = m.v_in(case["eta0"]), m.e_in(case["U0"])
    e2, u2 = e1, u1
    for _ in range(4):
        e1, u1, a1, _ = m.subcycle(e1, u1, volume=False, **kw)
        e2, u2, a2, _ = m.subcycle(e2, u2, volume=False, threads=0, **kw)
    assert m.threads_used >= 1
    assert np.array_equal(e1, e2) and np.array_equal(u1, u2) and np.array_equal(a1, a2)


def test_threaded_subcycle_refuses_viscous_term():
    case = sesynth.random_case(sesynth.tiny_mesh("jitter76"), seed=1, nsub=5)
    m = oracle.Mesh(case, reordered=True)
    with pytest.raises(ValueError):
        m.subcycle(m.v_in(case["eta0"]), m.e_in(case["U0"]), visc=(1.0, 0.0), threads=2,
                   **_inputs(case, m, False))
