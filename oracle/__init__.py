"""FP64 CPU oracle of the split-explicit barotropic subcycle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does, and
this package imports nothing from it.

Contents
  oracle.c     plain C definition (reorder, geometry, forward SE and SESM, TLM,
               adjoint, trim of layer transports and z* thicknesses, vertically
               integrated baroclinic forcing, barotropic viscous regularization)
  brute.py     dense operators from an independent median-dual construction
  analytic.py  closed forms of the paper's Sec. 3 (amplification matrix,
               characteristic polynomial, small-c expansions)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

PERIODIC_X, PERIODIC_Y, SPHERICAL = 1, 2, 4
_ERR = {1: "bad argument", 2: "invalid mesh", 3: "out of memory"}


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.orc_hilbert_d.restype = ctypes.c_uint64
        _lib.orc_hilbert_d.argtypes = [ctypes.c_uint32] * 3
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + _ERR.get(rc, str(rc)))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def forcing(*, K, nlev=None, RA=None, RP=None, RhV=None, tau_s=None, u=None, Cd=0.0):
    """Vertically integrated baroclinic forcing of eq. (eq4_4): per element the sum over
    its nlev layers of RA + RP + RhV, plus the surface stress tau_s, minus the bottom drag
    Cd |u_b| u_b on the velocity of the deepest layer.  Layer arrays [ne][K][2]."""
    L = _load()
    arrs = [a for a in (RA, RP, RhV, u) if a is not None]
    ne = np.asarray(arrs[0]).shape[0] if arrs else np.asarray(tau_s).shape[0]
    lay = lambda a: None if a is None else _f64(a, (ne, K, 2))
    nl = None if nlev is None else np.ascontiguousarray(nlev, np.int32)
    R = np.empty((ne, 2))
    _check(L.orc_forcing(ctypes.c_int64(ne), ctypes.c_int32(K), _p(nl), _p(lay(RA)), _p(lay(RP)),
                         _p(lay(RhV)), _p(None if tau_s is None else _f64(tau_s, (ne, 2))),
                         _p(lay(u)), ctypes.c_double(Cd), _p(R)))
    return R


def mesh_flags(mesh: dict) -> int:
    return ((PERIODIC_X if mesh.get("periodic_x") else 0) |
            (PERIODIC_Y if mesh.get("periodic_y") else 0) |
            (SPHERICAL if mesh.get("spherical") else 0))


def hilbert_d(side: int, x: int, y: int) -> int:
    return int(_load().orc_hilbert_d(side, x, y))


def reorder(mesh: dict):
    """(vperm, eperm, tri_new, row_ptr, col) exactly as the oracle defines them."""
    L = _load()
    x, y = _f64(mesh["x"]), _f64(mesh["y"])
    tri = np.ascontiguousarray(mesh["tri"], np.int32)
    nv, ne = x.size, tri.shape[0]
    vperm = np.empty(nv, np.int32)
    eperm = np.empty(ne, np.int32)
    tri_new = np.empty((ne, 3), np.int32)
    row_ptr = np.empty(nv + 1, np.int32)
    col = np.empty(3 * ne, np.int32)
    _check(L.orc_reorder(ctypes.c_int64(nv), ctypes.c_int64(ne), _p(x), _p(y), _p(tri),
                         _p(vperm), _p(eperm), _p(tri_new), _p(row_ptr), _p(col)))
    return vperm, eperm, tri_new, row_ptr, col


def geometry(mesh: dict, tri=None, x=None, y=None):
    """(Ae [ne], gN [ne,3,2], Av [nv]) for the mesh (or for a renumbered copy)."""
    L = _load()
    x = _f64(mesh["x"] if x is None else x)
    y = _f64(mesh["y"] if y is None else y)
    tri = np.ascontiguousarray(mesh["tri"] if tri is None else tri, np.int32)
    nv, ne = x.size, tri.shape[0]
    Ae = np.empty(ne)
    gN = np.empty((ne, 3, 2))
    Av = np.empty(nv)
    _check(L.orc_geometry(ctypes.c_int64(nv), ctypes.c_int64(ne), _p(x), _p(y), _p(tri),
                          ctypes.c_uint32(mesh_flags(mesh)), ctypes.c_double(mesh["period_x"]),
                          ctypes.c_double(mesh["period_y"]), ctypes.c_double(mesh["radius"]),
                          _p(Ae), _p(gN), _p(Av)))
    return Ae, gN, Av


class Mesh:
    """Oracle-side mesh: connectivity in some numbering plus FP64 geometry."""

    def __init__(self, mesh: dict, reordered: bool = True):
        self.src = mesh
        if reordered:
            self.vperm, self.eperm, self.tri, self.row_ptr, self.col = reorder(mesh)
            self.x = _f64(mesh["x"])[self.vperm]
            self.y = _f64(mesh["y"])[self.vperm]
        else:
            self.vperm = np.arange(mesh["x"].size, dtype=np.int32)
            self.eperm = np.arange(mesh["tri"].shape[0], dtype=np.int32)
            self.tri = np.ascontiguousarray(mesh["tri"], np.int32)
            self.x, self.y = _f64(mesh["x"]), _f64(mesh["y"])
        self.Ae, self.gN, self.Av = geometry(mesh, self.tri, self.x, self.y)
        self.nv, self.ne = self.x.size, self.tri.shape[0]

    # permutation helpers: original numbering <-> this mesh's numbering
    def v_in(self, a):
        return None if a is None else _f64(a)[self.vperm]

    def e_in(self, a):
        return None if a is None else np.ascontiguousarray(np.asarray(a, np.float64)[self.eperm])

    def v_out(self, a):
        out = np.empty_like(a)
        out[self.vperm] = a
        return out

    def e_out(self, a):
        out = np.empty_like(a)
        out[self.eperm] = a
        return out

    def _common(self, g, theta, linear_h, H0, f, R, W):
        return (ctypes.c_int64(self.nv), ctypes.c_int64(self.ne), _p(self.tri), _p(self.Ae),
                _p(self.gN), _p(self.Av), ctypes.c_double(g), ctypes.c_double(theta),
                ctypes.c_int(1 if linear_h else 0), _p(_f64(H0)), _p(_f64(f)),
                _p(_f64(R, (self.ne, 2))), _p(None if W is None else _f64(W)))

    def subcycle(self, eta, U, *, H0, f, R, W=None, g, theta, nsub, tau, linear_h=False,
                 volume=True, visc=None, threads=None):
        """One baroclinic step in this mesh's numbering.  Returns (eta, U, Uavg, volume).
        visc = (A0, Cv) adds the barotropic viscous regularization (eq. (eq:viscosity_BT))
        and subtracts its initial value from R.  threads = n (0: the OpenMP default) runs
        the multithreaded form (same eta, U, Uavg bit for bit; volume summed in fixed
        blocks); the thread count it used is left in self.threads_used."""
        L = _load()
        eta = _f64(eta).copy()
        U = _f64(U, (self.ne, 2)).copy()
        Uavg = np.empty((self.ne, 2))
        vol = np.empty(nsub + 1) if volume else None
        args = self._common(g, theta, linear_h, H0, f, R, W) + (
            ctypes.c_int32(nsub), ctypes.c_double(tau), _p(eta), _p(U), _p(Uavg), _p(vol))
        if threads is not None:
            if visc is not None:
                raise ValueError("oracle: the threaded subcycle has no viscous term")
            used = ctypes.c_int(0)
            _check(L.orc_subcycle_threads(*args, ctypes.c_int(threads), ctypes.byref(used)))
            self.threads_used = used.value
        elif visc is None:
            _check(L.orc_subcycle(*args))
        else:
            nb, elen, lod = self.visc_geometry()
            _check(L.orc_subcycle_visc(*args, _p(nb), _p(elen), _p(lod),
                                       ctypes.c_double(visc[0]), ctypes.c_double(visc[1])))
        return eta, U, Uavg, vol

    def visc_geometry(self):
        """(nb [ne][3], l [ne][3], l/d [ne][3]): the triangle across local edge j
        (t_j, t_{j+1}) or -1 on a coast, the edge length and the edge length over the
        distance between the two centroids."""
        if not hasattr(self, "_visc_geo"):
            L = _load()
            nb = np.empty((self.ne, 3), np.int32)
            _check(L.orc_edge_neighbours(ctypes.c_int64(self.ne), _p(self.tri), _p(nb)))
            elen = np.empty((self.ne, 3))
            lod = np.empty((self.ne, 3))
            m = self.src
            _check(L.orc_visc_geometry(ctypes.c_int64(self.nv), ctypes.c_int64(self.ne),
                                       _p(self.x), _p(self.y), _p(self.tri),
                                       ctypes.c_uint32(mesh_flags(m)),
                                       ctypes.c_double(m["period_x"]),
                                       ctypes.c_double(m["period_y"]),
                                       ctypes.c_double(m.get("radius", 0.0)), _p(nb), _p(elen),
                                       _p(lod)))
            self._visc_geo = (nb, elen, lod)
        return self._visc_geo

    def visc(self, eta, U, *, H0, A0, Cv, linear_h=False):
        """The barotropic viscous term R^hV(eta, U) of eq. (eq:viscosity_BT) [ne][2]."""
        L = _load()
        nb, elen, lod = self.visc_geometry()
        V = np.empty((self.ne, 2))
        _check(L.orc_visc_apply(ctypes.c_int64(self.nv), ctypes.c_int64(self.ne), _p(self.tri),
                                _p(self.Ae), _p(nb), _p(elen), _p(lod), ctypes.c_double(A0),
                                ctypes.c_double(Cv), ctypes.c_int(1 if linear_h else 0),
                                _p(_f64(H0)), _p(_f64(eta)), _p(_f64(U, (self.ne, 2))), _p(V)))
        return V

    def subcycle_sesm(self, eta, U, *, H0, f, R, W=None, g, beta, delta, gamma, zeta, nsub,
                      tau, linear_h=False, volume=True):
        """One baroclinic step of the AB3-AM4 (SESM) scheme, eqs. (eq4_7)-(eq4_8).
        Returns (eta, U, Uavg, volume); Uavg is the mean AB3 transport."""
        L = _load()
        eta = _f64(eta).copy()
        U = _f64(U, (self.ne, 2)).copy()
        Uavg = np.empty((self.ne, 2))
        vol = np.empty(nsub + 1) if volume else None
        args = (ctypes.c_int64(self.nv), ctypes.c_int64(self.ne), _p(self.tri), _p(self.Ae),
                _p(self.gN), _p(self.Av), ctypes.c_double(g), ctypes.c_double(beta),
                ctypes.c_double(delta), ctypes.c_double(gamma), ctypes.c_double(zeta),
                ctypes.c_int(1 if linear_h else 0), _p(_f64(H0)), _p(_f64(f)),
                _p(_f64(R, (self.ne, 2))), _p(None if W is None else _f64(W)),
                ctypes.c_int32(nsub), ctypes.c_double(tau), _p(eta), _p(U), _p(Uavg), _p(vol))
        _check(L.orc_subcycle_sesm(*args))
        return eta, U, Uavg, vol

    def trim_zstar(self, *, H0, eta_new, Uavg, Ustar, hn, h0, W=None, tau):
        """Trim of the layer transports to <<U>> (eq. (eq4_13)), z* thicknesses and the
        diasurface velocity.  Ustar [ne][K][2], hn/h0 [nv][K].  Returns (U, hnew, w[nv][K+1])."""
        L = _load()
        Ustar = np.ascontiguousarray(Ustar, np.float64)
        K = Ustar.shape[1]
        U = np.empty_like(Ustar)
        hnew = np.empty((self.nv, K))
        w = np.empty((self.nv, K + 1))
        _check(L.orc_trim_zstar(ctypes.c_int64(self.nv), ctypes.c_int64(self.ne), _p(self.tri),
                                _p(self.Ae), _p(self.gN), _p(self.Av), ctypes.c_int32(K),
                                _p(_f64(H0)), _p(_f64(eta_new)), _p(_f64(Uavg, (self.ne, 2))),
                                _p(Ustar), _p(_f64(hn, (self.nv, K))), _p(_f64(h0, (self.nv, K))),
                                _p(None if W is None else _f64(W)), ctypes.c_double(tau), _p(U),
                                _p(hnew), _p(w)))
        return U, hnew, w

    def tlm(self, eta0, U0, d_eta0, d_U0, d_R, d_H0, *, H0, f, R, W=None, g, theta, nsub,
            tau, linear_h=False):
        L = _load()
        d_eta = np.empty(self.nv)
        d_U = np.empty((self.ne, 2))
        d_Uavg = np.empty((self.ne, 2))
        _check(L.orc_tlm(*self._common(g, theta, linear_h, H0, f, R, W), ctypes.c_int32(nsub),
                         ctypes.c_double(tau), _p(_f64(eta0)), _p(_f64(U0, (self.ne, 2))),
                         _p(_f64(d_eta0)), _p(_f64(d_U0, (self.ne, 2))),
                         _p(_f64(d_R, (self.ne, 2))), _p(_f64(d_H0)), _p(d_eta), _p(d_U),
                         _p(d_Uavg)))
        return d_eta, d_U, d_Uavg

    def adjoint(self, eta0, U0, lam_eta=None, lam_U=None, lam_Uavg=None, *, H0, f, R, W=None,
                g, theta, nsub, tau, linear_h=False):
        """Gradients (eta0, U0, R, H0) of <lam_eta,eta^M> + <lam_U,U^M> + <lam_Uavg,Uavg>."""
        L = _load()
        g_eta0 = np.empty(self.nv)
        g_U0 = np.empty((self.ne, 2))
        g_R = np.empty((self.ne, 2))
        g_H0 = np.empty(self.nv)
        _check(L.orc_adjoint(*self._common(g, theta, linear_h, H0, f, R, W),
                             ctypes.c_int32(nsub), ctypes.c_double(tau), _p(_f64(eta0)),
                             _p(_f64(U0, (self.ne, 2))),
                             _p(None if lam_eta is None else _f64(lam_eta)),
                             _p(None if lam_U is None else _f64(lam_U, (self.ne, 2))),
                             _p(None if lam_Uavg is None else _f64(lam_Uavg, (self.ne, 2))),
                             _p(g_eta0), _p(g_U0), _p(g_R), _p(g_H0)))
        return g_eta0, g_U0, g_R, g_H0


def run_case(case: dict, nsteps: int | None = None, reordered: bool = True, mesh: Mesh = None,
             threads=None):
    """Run a generated workload through the oracle, in the oracle's reordered numbering
    (threads: see Mesh.subcycle).

    Returns dict(mesh, eta, U, Uavg (last step), volume (all substeps), inputs...).
    """
    m = mesh if mesh is not None else Mesh(case, reordered=reordered)
    H0, f, R = m.v_in(case["H0"]), m.e_in(case["f"]), m.e_in(case["R"])
    W = m.v_in(case["W"]) if case.get("W") is not None else None
    eta, U = m.v_in(case["eta0"]), m.e_in(case["U0"])
    nsteps = case["nsteps"] if nsteps is None else nsteps
    vols = []
    Uavg = None
    for _ in range(nsteps):
        eta, U, Uavg, vol = m.subcycle(eta, U, H0=H0, f=f, R=R, W=W, g=case["g"],
                                       theta=case["theta"], nsub=case["nsub"],
                                       tau=case["tau"], linear_h=case["linear_h"],
                                       threads=threads)
        vols.append(vol if not vols else vol[1:])
    return dict(mesh=m, eta=eta, U=U, Uavg=Uavg, volume=np.concatenate(vols), H0=H0, f=f, R=R)
