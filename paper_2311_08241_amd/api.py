"""Python face of the C ABI: the same entry points, argument marshalling only.

torch provides device memory and streams; every step of the subcycle runs in
libsesub.so.  Field tensors are in the mesh's internal (reordered) numbering;
Mesh.v_in / e_in / v_out / e_out convert from and to the caller's numbering.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def sesm_coefficients(theta: float = 0.14, beta: float = 0.0):
    """(beta, delta, gamma, zeta) of the AB3-AM4 scheme at the dissipation of the
    forward-backward scheme with this theta (se_sesm_coefficients)."""
    out = (ctypes.c_double * 4)()
    L.check(L.lib().se_sesm_coefficients(float(theta), float(beta), out))
    return tuple(out)


@dataclass
class Params:
    """se_params: g, theta (eq. (eq4_10)), precision, flags, eta_ref, h_max, scheme
    ("se" or "sesm", eqs. (eq4_7)-(eq4_8)), the SESM coefficients (default: those
    of sesm_coefficients(theta)) and the barotropic viscous regularization
    visc = (A0, Cv) of eq. (eq:viscosity_BT) (plain SE path only)."""
    g: float = 9.81
    theta: float = 0.14
    precision: str = "f64"          # "f64" | "f32" (FP32 bulk, FP64 volume and average)
    linear_h: bool = False
    check_cfl: bool = False
    track_volume: bool = True
    eta_ref: float = 0.0
    h_max: float = 0.0
    scheme: str = "se"
    sesm: tuple | None = None       # (beta, delta, gamma, zeta)
    visc: tuple | None = None       # (A0, Cv): background and flow-dependent coefficients

    @property
    def dtype(self):
        torch = _torch()
        return torch.float64 if self.precision == "f64" else torch.float32

    def c(self) -> L.Params:
        if self.precision not in ("f64", "f32"):
            raise ValueError("precision must be 'f64' or 'f32'")
        flags = ((L.SE_LINEAR_H if self.linear_h else 0) |
                 (L.SE_CHECK_CFL if self.check_cfl else 0) |
                 (L.SE_TRACK_VOLUME if self.track_volume else 0))
        if self.scheme not in ("se", "sesm"):
            raise ValueError("scheme must be 'se' or 'sesm'")
        co = (self.sesm if self.sesm is not None else sesm_coefficients(self.theta)) \
            if self.scheme == "sesm" else (0.0, 0.0, 0.0, 0.0)
        return L.Params(self.g, self.theta,
                        L.SE_F64 if self.precision == "f64" else L.SE_F32_MIXED, flags,
                        self.eta_ref, self.h_max,
                        L.SE_SCHEME_SESM if self.scheme == "sesm" else L.SE_SCHEME_SE, 0,
                        *[float(v) for v in co],
                        *([0.0, 0.0] if self.visc is None else [float(v) for v in self.visc]))


class Mesh:
    """A reordered mesh owned by the library (se_mesh_create)."""

    def __init__(self, x, y, tri, *, periodic_x=False, periodic_y=False, period_x=0.0,
                 period_y=0.0, spherical=False, radius=0.0, device: int = 0):
        self._x = np.ascontiguousarray(x, np.float64)
        self._y = np.ascontiguousarray(y, np.float64)
        self._tri = np.ascontiguousarray(tri, np.int32)
        flags = ((L.SE_PERIODIC_X if periodic_x else 0) | (L.SE_PERIODIC_Y if periodic_y else 0) |
                 (L.SE_SPHERICAL if spherical else 0))
        d = L.MeshDesc(self._x.size, self._tri.shape[0],
                       self._x.ctypes.data_as(ctypes.c_void_p),
                       self._y.ctypes.data_as(ctypes.c_void_p),
                       self._tri.ctypes.data_as(ctypes.c_void_p), flags, float(period_x),
                       float(period_y), float(radius))
        h = ctypes.c_void_p()
        L.check(L.lib().se_mesh_create(ctypes.byref(d), int(device), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        nv, ne, nnz, mu = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        L.check(L.lib().se_mesh_info(h, ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(nnz),
                                     ctypes.byref(mu)))
        self.nv, self.ne, self.nnz, self.mu_max = nv.value, ne.value, nnz.value, mu.value
        self.vperm = np.empty(self.nv, np.int32)
        self.eperm = np.empty(self.ne, np.int32)
        L.check(L.lib().se_mesh_perm(h, self.vperm.ctypes.data_as(ctypes.c_void_p),
                                     self.eperm.ctypes.data_as(ctypes.c_void_p)))

    @classmethod
    def from_dict(cls, m: dict, device: int = 0):
        return cls(m["x"], m["y"], m["tri"], periodic_x=m.get("periodic_x", False),
                   periodic_y=m.get("periodic_y", False), period_x=m.get("period_x", 0.0),
                   period_y=m.get("period_y", 0.0), spherical=m.get("spherical", False),
                   radius=m.get("radius", 0.0), device=device)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().se_mesh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- host copies ----
    def csr(self):
        tri = np.empty((self.ne, 3), np.int32)
        row = np.empty(self.nv + 1, np.int32)
        col = np.empty(self.nnz, np.int32)
        L.check(L.lib().se_mesh_csr(self._h, tri.ctypes.data_as(ctypes.c_void_p),
                                    row.ctypes.data_as(ctypes.c_void_p),
                                    col.ctypes.data_as(ctypes.c_void_p)))
        return tri, row, col

    def geometry(self):
        Av = np.empty(self.nv)
        Ae = np.empty(self.ne)
        gN = np.empty((self.ne, 3, 2))
        L.check(L.lib().se_mesh_geometry(self._h, Av.ctypes.data_as(ctypes.c_void_p),
                                         Ae.ctypes.data_as(ctypes.c_void_p),
                                         gN.ctypes.data_as(ctypes.c_void_p)))
        return Av, Ae, gN

    def neighbours(self):
        """(nb [ne][3], l [ne][3], l/d [ne][3]) of the barotropic viscous term."""
        nb = np.empty((self.ne, 3), np.int32)
        ln = np.empty((self.ne, 3))
        lod = np.empty((self.ne, 3))
        L.check(L.lib().se_mesh_neighbours(self._h, nb.ctypes.data_as(ctypes.c_void_p),
                                           ln.ctypes.data_as(ctypes.c_void_p),
                                           lod.ctypes.data_as(ctypes.c_void_p)))
        return nb, ln, lod

    # ---- numbering helpers (caller numbering <-> internal) ----
    def v_in(self, a):
        return np.ascontiguousarray(np.asarray(a)[self.vperm])

    def e_in(self, a):
        return np.ascontiguousarray(np.asarray(a)[self.eperm])

    def v_out(self, a):
        out = np.empty_like(a)
        out[self.vperm] = a
        return out

    def e_out(self, a):
        out = np.empty_like(a)
        out[self.eperm] = a
        return out

    # ---- plan ----
    def set_plan(self, tile: int, k_fused: int, block: int = 256):
        L.check(L.lib().se_set_plan(self._h, 0, int(tile), int(k_fused), int(block)))

    def plan_stats(self, tile: int, k_fused: int, block: int = 256) -> dict:
        st = L.PlanStats()
        L.check(L.lib().se_plan_stats(self._h, 0, int(tile), int(k_fused), int(block),
                                      ctypes.byref(st)))
        return st.as_dict()

    def get_plan(self):
        t, k, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().se_get_plan(self._h, 0, ctypes.byref(t), ctypes.byref(k), ctypes.byref(b)))
        return t.value, k.value, b.value

    # ---- compute ----
    def workspace_bytes(self, params: Params, nsub: int, ckpt_every: int = 0) -> int:
        n = ctypes.c_size_t()
        pc = params.c()
        L.check(L.lib().se_workspace_bytes(self._h, ctypes.byref(pc), int(nsub), int(ckpt_every),
                                           ctypes.byref(n)))
        return n.value

    def workspace(self, params: Params, nsub: int, ckpt_every: int = 0):
        torch = _torch()
        n = self.workspace_bytes(params, nsub, ckpt_every)
        # torch's caching allocator returns 256-byte aligned blocks
        return torch.empty(max(n, 256), dtype=torch.uint8, device=f"cuda:{self.device}")

    def _check_tensor(self, t, n, name, dtype, cols=None, allow_none=False):
        if t is None:
            if allow_none:
                return
            raise ValueError(f"{name} is required")
        shape = (n,) if cols is None else (n, cols)
        if tuple(t.shape) != shape or t.dtype != dtype or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of shape {shape}, "
                             f"got {tuple(t.shape)} {t.dtype} cuda={t.is_cuda}")

    def subcycle(self, eta, U, *, R, f, H0, W=None, nsub: int, dt: float, params: Params,
                 Uavg=None, volume=None, workspace=None, plain: bool = False, stream=None):
        """se_subcycle (or se_subcycle_plain): eta, U updated in place; fills Uavg, volume."""
        torch = _torch()
        dt_ = params.dtype
        self._check_tensor(eta, self.nv, "eta", dt_)
        self._check_tensor(U, self.ne, "U", dt_, 2)
        self._check_tensor(R, self.ne, "R", dt_, 2)
        self._check_tensor(f, self.ne, "f", dt_)
        self._check_tensor(H0, self.nv, "H0", dt_)
        self._check_tensor(W, self.nv, "W", dt_, allow_none=True)
        self._check_tensor(Uavg, self.ne, "Uavg", torch.float64, 2, allow_none=True)
        nvol = nsub + 1 if params.track_volume else 2
        self._check_tensor(volume, nvol, "volume", torch.float64, allow_none=True)
        if workspace is None:
            workspace = self.workspace(params, nsub)
        st = L.State(_ptr(eta), _ptr(U), _ptr(Uavg), _ptr(volume))
        fo = L.Forcing(_ptr(R), _ptr(f), _ptr(H0), _ptr(W))
        pc = params.c()
        fn = L.lib().se_subcycle_plain if plain else L.lib().se_subcycle
        L.check(fn(self._h, ctypes.byref(pc), ctypes.byref(st), ctypes.byref(fo), int(nsub),
                   float(dt), _ptr(workspace), _stream_ptr(stream)))
        return eta, U, Uavg, volume

    def subcycle_noalloc(self, eta, U, *, R, f, H0, W=None, nsub: int, dt: float,
                         params: Params, Uavg=None, volume=None, stream=None):
        """se_subcycle_noalloc: se_subcycle with the library's static device scratch as
        workspace (nothing allocated; the mesh needs a tile plan already)."""
        torch = _torch()
        dt_ = params.dtype
        self._check_tensor(eta, self.nv, "eta", dt_)
        self._check_tensor(U, self.ne, "U", dt_, 2)
        self._check_tensor(R, self.ne, "R", dt_, 2)
        self._check_tensor(f, self.ne, "f", dt_)
        self._check_tensor(H0, self.nv, "H0", dt_)
        self._check_tensor(W, self.nv, "W", dt_, allow_none=True)
        self._check_tensor(Uavg, self.ne, "Uavg", torch.float64, 2, allow_none=True)
        nvol = nsub + 1 if params.track_volume else 2
        self._check_tensor(volume, nvol, "volume", torch.float64, allow_none=True)
        st = L.State(_ptr(eta), _ptr(U), _ptr(Uavg), _ptr(volume))
        fo = L.Forcing(_ptr(R), _ptr(f), _ptr(H0), _ptr(W))
        pc = params.c()
        L.check(L.lib().se_subcycle_noalloc(self._h, ctypes.byref(pc), ctypes.byref(st),
                                            ctypes.byref(fo), int(nsub), float(dt),
                                            _stream_ptr(stream)))
        return eta, U, Uavg, volume

    def trim_zstar(self, *, H0, eta_new, Uavg, Ustar, hn, h0, tau: float, W=None, U=None,
                   hnew=None, w=None, stream=None):
        """se_trim_zstar (FP64): trim of the layer transports Ustar [ne][K][2] to Uavg
        (eq. (eq4_13)), z* thicknesses and the diasurface velocity.  Outputs that are
        None are allocated (U may be Ustar itself).  Returns (U, hnew, w)."""
        torch = _torch()
        f64 = torch.float64
        K = int(Ustar.shape[1])
        for t, n, name in ((H0, self.nv, "H0"), (eta_new, self.nv, "eta_new")):
            self._check_tensor(t, n, name, f64)
        self._check_tensor(Uavg, self.ne, "Uavg", f64, 2)
        self._check_tensor(W, self.nv, "W", f64, allow_none=True)
        if tuple(Ustar.shape) != (self.ne, K, 2) or Ustar.dtype != f64 or not Ustar.is_contiguous():
            raise ValueError("Ustar must be a contiguous float64 tensor [ne][K][2]")
        for t, name in ((hn, "hn"), (h0, "h0")):
            if tuple(t.shape) != (self.nv, K) or t.dtype != f64 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 tensor [nv][K]")
        dev = Ustar.device
        U = torch.empty_like(Ustar) if U is None else U
        hnew = torch.empty((self.nv, K), dtype=f64, device=dev) if hnew is None else hnew
        w = torch.empty((self.nv, K + 1), dtype=f64, device=dev) if w is None else w
        L.check(L.lib().se_trim_zstar(self._h, K, _ptr(H0), _ptr(eta_new), _ptr(Uavg),
                                      _ptr(Ustar), _ptr(hn), _ptr(h0), _ptr(W), float(tau),
                                      _ptr(U), _ptr(hnew), _ptr(w), _stream_ptr(stream)))
        return U, hnew, w

    def visc(self, eta, U, *, H0, A0: float, Cv: float, precision: str = "f64",
             linear_h: bool = False, eta_ref: float = 0.0, V=None, workspace=None, stream=None):
        """se_barotropic_visc: the barotropic viscous term R^hV(eta, U) of
        eq. (eq:viscosity_BT) per triangle, [ne][2] in the precision's dtype."""
        torch = _torch()
        dt = torch.float64 if precision == "f64" else torch.float32
        if precision not in ("f64", "f32"):
            raise ValueError("precision must be 'f64' or 'f32'")
        self._check_tensor(H0, self.nv, "H0", dt)
        self._check_tensor(eta, self.nv, "eta", dt)
        self._check_tensor(U, self.ne, "U", dt, 2)
        V = torch.empty((self.ne, 2), dtype=dt, device=U.device) if V is None else V
        self._check_tensor(V, self.ne, "V", dt, 2)
        ws = torch.empty((self.ne, 2), dtype=dt, device=U.device) if workspace is None \
            else workspace
        L.check(L.lib().se_barotropic_visc(self._h, L.SE_F64 if precision == "f64" else
                                           L.SE_F32_MIXED, L.SE_LINEAR_H if linear_h else 0,
                                           float(eta_ref), float(A0), float(Cv), _ptr(H0),
                                           _ptr(eta), _ptr(U), _ptr(V), _ptr(ws),
                                           _stream_ptr(stream)))
        return V

    def forcing(self, *, K: int, nlev=None, RA=None, RP=None, RhV=None, tau_s=None, u=None,
                Cd: float = 0.0, precision: str = "f64", R=None, stream=None):
        """se_forcing_assemble: vertically integrated baroclinic forcing of eq. (eq4_4) per triangle,
        the sum over its nlev layers of RA + RP + RhV ([ne][K][2] float64 each, any may be
        None), plus the surface stress tau_s [ne][2], minus Cd |u_b| u_b on the deepest
        layer's velocity u [ne][K][2].  Returns R [ne][2] (float64, or float32 for
        precision "f32", the FP32 subcycle's forcing)."""
        torch = _torch()
        f64 = torch.float64
        K = int(K)
        for t, name in ((RA, "RA"), (RP, "RP"), (RhV, "RhV"), (u, "u")):
            if t is not None and (tuple(t.shape) != (self.ne, K, 2) or t.dtype != f64
                                  or not t.is_contiguous() or not t.is_cuda):
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor [ne][K][2]")
        self._check_tensor(tau_s, self.ne, "tau_s", f64, 2, allow_none=True)
        if nlev is not None and (tuple(nlev.shape) != (self.ne,) or nlev.dtype != torch.int32
                                 or not nlev.is_contiguous() or not nlev.is_cuda):
            raise ValueError("nlev must be a contiguous int32 CUDA tensor [ne]")
        if precision not in ("f64", "f32"):
            raise ValueError("precision must be 'f64' or 'f32'")
        dt = f64 if precision == "f64" else torch.float32
        if R is None:
            dev = next(t.device for t in (RA, RP, RhV, u, tau_s, nlev) if t is not None)
            R = torch.empty((self.ne, 2), dtype=dt, device=dev)
        self._check_tensor(R, self.ne, "R", dt, 2)
        L.check(L.lib().se_forcing_assemble(self._h, K, _ptr(nlev), _ptr(RA), _ptr(RP), _ptr(RhV),
                                   _ptr(tau_s), _ptr(u), float(Cd),
                                   L.SE_F64 if precision == "f64" else L.SE_F32_MIXED, _ptr(R),
                                   _stream_ptr(stream)))
        return R

    def adjoint(self, eta0, U0, *, R, f, H0, W=None, nsub: int, dt: float, params: Params,
                ckpt_every: int = 5, lam_eta=None, lam_U=None, lam_Uavg=None, g_eta0=None,
                g_U0=None, g_R=None, g_H0=None, workspace=None, stream=None):
        """se_subcycle_adjoint: gradients of <lam_eta, eta^M> + <lam_U, U^M> + <lam_Uavg, <<U>>>.

        Outputs that are None are allocated; returns (g_eta0, g_U0, g_R, g_H0).
        """
        torch = _torch()
        dt_ = params.dtype
        dev = f"cuda:{self.device}"
        for t, n, name, cols in ((eta0, self.nv, "eta0", None), (U0, self.ne, "U0", 2),
                                 (R, self.ne, "R", 2), (f, self.ne, "f", None),
                                 (H0, self.nv, "H0", None)):
            self._check_tensor(t, n, name, dt_, cols)
        self._check_tensor(W, self.nv, "W", dt_, allow_none=True)
        self._check_tensor(lam_eta, self.nv, "lam_eta", dt_, allow_none=True)
        self._check_tensor(lam_U, self.ne, "lam_U", dt_, 2, allow_none=True)
        self._check_tensor(lam_Uavg, self.ne, "lam_Uavg", torch.float64, 2, allow_none=True)
        g_eta0 = torch.empty(self.nv, dtype=dt_, device=dev) if g_eta0 is None else g_eta0
        g_U0 = torch.empty((self.ne, 2), dtype=dt_, device=dev) if g_U0 is None else g_U0
        g_R = torch.empty((self.ne, 2), dtype=dt_, device=dev) if g_R is None else g_R
        g_H0 = torch.empty(self.nv, dtype=dt_, device=dev) if g_H0 is None else g_H0
        self._check_tensor(g_eta0, self.nv, "g_eta0", dt_)
        self._check_tensor(g_U0, self.ne, "g_U0", dt_, 2)
        self._check_tensor(g_R, self.ne, "g_R", dt_, 2)
        self._check_tensor(g_H0, self.nv, "g_H0", dt_)
        if workspace is None:
            workspace = self.workspace(params, nsub, ckpt_every)
        fo = L.Forcing(_ptr(R), _ptr(f), _ptr(H0), _ptr(W))
        pc = params.c()
        L.check(L.lib().se_subcycle_adjoint(
            self._h, ctypes.byref(pc), _ptr(eta0), _ptr(U0), ctypes.byref(fo), int(nsub),
            float(dt), int(ckpt_every), _ptr(lam_eta), _ptr(lam_U), _ptr(lam_Uavg),
            _ptr(g_eta0), _ptr(g_U0), _ptr(g_R), _ptr(g_H0), _ptr(workspace),
            _stream_ptr(stream)))
        return g_eta0, g_U0, g_R, g_H0

    def check_faults(self, stream=None) -> int:
        bits = ctypes.c_uint32()
        L.check(L.lib().se_check_faults(self._h, 0, _stream_ptr(stream), ctypes.byref(bits)))
        return bits.value


class Batch:
    """Ensemble of independent meshes advanced together (se_batch_create).

    Field tensors are the members' internal-numbering arrays concatenated in
    member order (vertex arrays at vert_offset, triangle arrays at elem_offset).
    """

    def __init__(self, meshes):
        self.meshes = list(meshes)
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = ctypes.c_void_p()
        L.check(L.lib().se_batch_create(arr, len(self.meshes), ctypes.byref(h)))
        self._h = h
        self.device = self.meshes[0].device
        n = len(self.meshes)
        nv, ne = ctypes.c_int64(), ctypes.c_int64()
        vo = (ctypes.c_int64 * (n + 1))()
        eo = (ctypes.c_int64 * (n + 1))()
        L.check(L.lib().se_batch_info(h, ctypes.byref(nv), ctypes.byref(ne), vo, eo))
        self.nv, self.ne = nv.value, ne.value
        self.vert_offset = np.array(vo[:], np.int64)
        self.elem_offset = np.array(eo[:], np.int64)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().se_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def signature(self) -> str:
        from .autotune import mesh_signature
        return "+".join(mesh_signature(m) for m in self.meshes)

    def set_plan(self, tile: int, k_fused: int, block: int = 256):
        L.check(L.lib().se_set_plan(self._h, 1, int(tile), int(k_fused), int(block)))

    def get_plan(self):
        t, k, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().se_get_plan(self._h, 1, ctypes.byref(t), ctypes.byref(k), ctypes.byref(b)))
        return t.value, k.value, b.value

    def plan_stats(self, tile: int, k_fused: int, block: int = 256) -> dict:
        st = L.PlanStats()
        L.check(L.lib().se_plan_stats(self._h, 1, int(tile), int(k_fused), int(block),
                                      ctypes.byref(st)))
        return st.as_dict()

    def volume_size(self, params: Params, nsub) -> int:
        return int(sum((k + 1) if params.track_volume else 2 for k in nsub))

    def workspace(self, params: Params, nsub):
        torch = _torch()
        ns = (ctypes.c_int32 * len(nsub))(*[int(k) for k in nsub])
        n = ctypes.c_size_t()
        pc = params.c()
        L.check(L.lib().se_batch_workspace_bytes(self._h, ctypes.byref(pc), ns, ctypes.byref(n)))
        return torch.empty(max(n.value, 256), dtype=torch.uint8, device=f"cuda:{self.device}")

    def subcycle(self, eta, U, *, R, f, H0, W=None, nsub, dt, params: Params, Uavg=None,
                 volume=None, workspace=None, use_graph=False, stream=None):
        """se_subcycle_batched: one baroclinic step of every member."""
        torch = _torch()
        dt_ = params.dtype
        chk = Mesh._check_tensor
        chk(self, eta, self.nv, "eta", dt_)
        chk(self, U, self.ne, "U", dt_, 2)
        chk(self, R, self.ne, "R", dt_, 2)
        chk(self, f, self.ne, "f", dt_)
        chk(self, H0, self.nv, "H0", dt_)
        chk(self, W, self.nv, "W", dt_, allow_none=True)
        chk(self, Uavg, self.ne, "Uavg", torch.float64, 2, allow_none=True)
        chk(self, volume, self.volume_size(params, nsub), "volume", torch.float64, allow_none=True)
        if len(nsub) != len(self.meshes) or len(dt) != len(self.meshes):
            raise ValueError("nsub and dt need one entry per member")
        if workspace is None:
            workspace = self.workspace(params, nsub)
        ns = (ctypes.c_int32 * len(nsub))(*[int(k) for k in nsub])
        dts = (ctypes.c_double * len(dt))(*[float(v) for v in dt])
        st = L.State(_ptr(eta), _ptr(U), _ptr(Uavg), _ptr(volume))
        fo = L.Forcing(_ptr(R), _ptr(f), _ptr(H0), _ptr(W))
        pc = params.c()
        L.check(L.lib().se_subcycle_batched(self._h, ctypes.byref(pc), ctypes.byref(st),
                                            ctypes.byref(fo), ns, dts, int(bool(use_graph)),
                                            _ptr(workspace), _stream_ptr(stream)))
        return eta, U, Uavg, volume

    def check_faults(self, stream=None) -> int:
        bits = ctypes.c_uint32()
        L.check(L.lib().se_check_faults(self._h, 1, _stream_ptr(stream), ctypes.byref(bits)))
        return bits.value


def batch_inputs(batch: Batch, cases, params: Params):
    """Concatenate generated member workloads into device tensors (internal numbering)."""
    parts = [device_inputs(m, c, params) for m, c in zip(batch.meshes, cases)]
    torch = _torch()
    out = {}
    for k in ("eta", "U", "R", "f", "H0"):
        out[k] = torch.cat([p[k] for p in parts]).contiguous()
    out["W"] = None
    return out


def device_inputs(mesh: Mesh, case: dict, params: Params, device=None):
    """Move a generated workload's fields to the device in the mesh's numbering.

    Returns dict(eta, U, R, f, H0, W) of tensors with params.dtype; eta holds
    eta - eta_ref in the FP32 mode.
    """
    torch = _torch()
    dev = device or f"cuda:{mesh.device}"
    dt_ = params.dtype
    eta = mesh.v_in(case["eta0"])
    if params.precision == "f32":
        eta = eta - params.eta_ref
    out = dict(
        eta=torch.tensor(eta, dtype=dt_, device=dev),
        U=torch.tensor(mesh.e_in(case["U0"]), dtype=dt_, device=dev).contiguous(),
        R=torch.tensor(mesh.e_in(case["R"]), dtype=dt_, device=dev).contiguous(),
        f=torch.tensor(mesh.e_in(case["f"]), dtype=dt_, device=dev),
        H0=torch.tensor(mesh.v_in(case["H0"]), dtype=dt_, device=dev),
        W=None if case.get("W") is None else torch.tensor(mesh.v_in(case["W"]), dtype=dt_,
                                                          device=dev),
    )
    return out
