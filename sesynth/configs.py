"""Seeded synthetic workloads for the barotropic subcycle.

Each builder returns a dict holding the mesh (see :mod:`sesynth.meshes`) and
the inputs of one run, all in the generator's own (unreordered) numbering:

    H0   float64 [nv]     resting depth at vertices (m)
    f    float64 [ne]     Coriolis parameter per triangle (1/s)
    R    float64 [ne, 2]  frozen barotropic forcing per triangle (m^2/s^2)
    eta0 float64 [nv]     initial elevation (m)
    U0   float64 [ne, 2]  initial depth-integrated transport (m^2/s)
    W    None             freshwater flux (zero in every workload)
    g, theta, tau, nsub, nsteps, linear_h, eta_ref   run parameters

The workloads stand in for the paper's channel and global experiments, whose
meshes and atmospheric forcing are not available; they keep the shapes, sizes
and value ranges and nothing else.  None of this code evaluates the scheme.
"""
from __future__ import annotations

import numpy as np

from . import meshes as M

G = 9.81
THETA = 0.14
OMEGA = 7.2921e-5
# |lambda| <= 1 for the dissipative forward-backward step iff c <= 2/sqrt(1+2 theta)
# (used here only to pick substep lengths for the generated ensembles).
_C_STAB = 2.0 / np.sqrt(1.0 + 2.0 * THETA)


def _blobs(px, py, r, nblob, lx, ly, smin, smax, periodic_x):
    """Sum of nblob Gaussian bumps with weights U(0.5, 1) and widths U(smin, smax)."""
    cx = r.uniform(0.0, lx, nblob)
    cy = r.uniform(0.0, ly, nblob)
    a = r.uniform(0.5, 1.0, nblob)
    s = r.uniform(smin, smax, nblob)
    out = np.zeros_like(px)
    for k in range(nblob):
        dx = px - cx[k]
        if periodic_x:
            dx = dx - lx * np.round(dx / lx)
        dy = py - cy[k]
        out += a[k] * np.exp(-(dx * dx + dy * dy) / (2.0 * s[k] * s[k]))
    return out


def _signed_blobs(px, py, r, nblob, lx, ly, smin, smax, periodic_x):
    cx = r.uniform(0.0, lx, nblob)
    cy = r.uniform(0.0, ly, nblob)
    a = r.standard_normal(nblob)
    s = r.uniform(smin, smax, nblob)
    out = np.zeros_like(px)
    for k in range(nblob):
        dx = px - cx[k]
        if periodic_x:
            dx = dx - lx * np.round(dx / lx)
        dy = py - cy[k]
        out += a[k] * np.exp(-(dx * dx + dy * dy) / (2.0 * s[k] * s[k]))
    return out


def _normalize01(v):
    return (v - v.min()) / max(v.max() - v.min(), 1e-300)


def _rms_scale(v, target):
    rms = np.sqrt(np.mean(v * v))
    return v * (target / max(rms, 1e-300))


def _smooth_noise(r, shape, sigma, wrap_x=True):
    """Gaussian-filtered white noise, unit variance, statistically uniform up to the edges.

    The noise is drawn on a grid padded by 3 sigma on every non-periodic side and
    cropped after filtering, so edge rows are no rougher or larger than the interior.
    """
    from scipy.ndimage import gaussian_filter
    pad = int(np.ceil(3 * sigma))
    ny, nx = shape
    px = 0 if wrap_x else pad
    z = r.standard_normal((ny + 2 * pad, nx + 2 * px))
    z = gaussian_filter(z, sigma=sigma, mode=("nearest", "wrap" if wrap_x else "nearest"))
    z = z[pad:pad + ny, px:px + nx]
    z = z - z.mean()
    return z / max(z.std(), 1e-300)


def _elem_mean(vfield, tri):
    return vfield[tri].mean(axis=1)


def _gaussian_eta(mesh, r, amp, sig_cells):
    """Gaussian bump of the given amplitude, width sig_cells grid cells, random centre."""
    nx, ny, dx, dy = mesh["nx"], mesh["ny"], mesh["dx"], mesh["dy"]
    sx, sy = sig_cells * dx, sig_cells * dy
    lx, ly = (nx - 1) * dx, (ny - 1) * dy
    cx = r.uniform(2 * sx, max(lx - 2 * sx, 2 * sx + 1e-9))
    cy = r.uniform(2 * sy, max(ly - 2 * sy, 2 * sy + 1e-9))
    ddx = mesh["x"] - cx
    if mesh["periodic_x"]:
        px = mesh["period_x"]
        ddx = ddx - px * np.round(ddx / px)
    ddy = mesh["y"] - cy
    return amp * np.exp(-0.5 * ((ddx / sx) ** 2 + (ddy / sy) ** 2))


def _pack(mesh, H0, f, R, eta0, U0, *, tau, nsub, nsteps, name, linear_h=False,
          g=G, theta=THETA, eta_ref=None):
    ne = mesh["tri"].shape[0]
    if U0 is None:
        U0 = np.zeros((ne, 2))
    if eta_ref is None:
        eta_ref = float(np.mean(eta0))
    d = dict(mesh)
    d.update(name=name, H0=np.ascontiguousarray(H0, np.float64),
             f=np.ascontiguousarray(f, np.float64),
             R=np.ascontiguousarray(R, np.float64).reshape(ne, 2),
             eta0=np.ascontiguousarray(eta0, np.float64),
             U0=np.ascontiguousarray(U0, np.float64).reshape(ne, 2), W=None,
             g=float(g), theta=float(theta), tau=float(tau), nsub=int(nsub),
             nsteps=int(nsteps), linear_h=bool(linear_h), eta_ref=float(eta_ref))
    return d


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def basin_c1(seed: int = 0):
    """Closed 64x32 basin, 2000 km x 1000 km, flat 4000 m, f = 1e-4, Gaussian bump."""
    r = M.rng(100 + seed)
    nx, ny = 64, 32
    mesh = M.planar_grid(nx, ny, 2.0e6 / (nx - 1), 1.0e6 / (ny - 1))
    nv, ne = mesh["x"].size, mesh["tri"].shape[0]
    eta0 = _gaussian_eta(mesh, r, 1.0, 5.0)
    return _pack(mesh, np.full(nv, 4000.0), np.full(ne, 1.0e-4), np.zeros((ne, 2)),
                 eta0, None, tau=900.0, nsub=30, nsteps=20, name="C1-basin-64x32")


def channel_c2(seed: int = 0, nx: int = 1024, ny: int = 512, delta: float = 2000.0,
               nsteps: int = 50):
    """x-periodic beta-plane channel, jittered, sum-of-64-Gaussians bathymetry."""
    r = M.rng(200 + seed)
    mesh = M.planar_grid(nx, ny, delta, delta, periodic_x=True, jitter=0.3, r=r)
    lx, ly = nx * delta, (ny - 1) * delta
    hb = _blobs(mesh["x"], mesh["y"], r, 64, lx, ly, 40e3, 300e3, True)
    H0 = 100.0 + 4900.0 * _normalize01(hb)
    cx, cy = M.element_centroid_planar(mesh)
    f = 1.0e-4 + 2.0e-11 * cy
    ax = _rms_scale(_signed_blobs(cx, cy, r, 64, lx, ly, 40e3, 300e3, True), 1.0e-5)
    ay = _rms_scale(_signed_blobs(cx, cy, r, 64, lx, ly, 40e3, 300e3, True), 1.0e-5)
    He = _elem_mean(H0, mesh["tri"])
    R = np.stack([He * ax, He * ay], -1)
    eta0 = _gaussian_eta(mesh, r, 1.0, 20.0)
    return _pack(mesh, H0, f, R, eta0, None, tau=180.0, nsub=60, nsteps=nsteps,
                 name=f"C2-channel-{nx}x{ny}")


def latlon_c3(seed: int = 0, nlon: int = 2048, nlat: int = 1536, nsteps: int = 20,
              land_fraction: float = 0.30):
    """Global-like lat-lon mesh over [-72, 72] deg with a seeded 30% land mask."""
    r = M.rng(300 + seed)
    full = M.latlon_grid(nlon, nlat, -72.0, 72.0)
    land_noise = _smooth_noise(r, (nlat, nlon), 16.0).ravel()
    wet = land_noise > np.quantile(land_noise, land_fraction)
    zH = _smooth_noise(r, (nlat, nlon), 8.0).ravel()
    H0_full = np.clip(np.exp(np.log(3500.0) + 0.9 * zH), 10.0, 6000.0)
    ax_full = _smooth_noise(r, (nlat, nlon), 16.0).ravel()
    ay_full = _smooth_noise(r, (nlat, nlon), 16.0).ravel()
    eta_full = 0.5 * _smooth_noise(r, (nlat, nlon), 16.0).ravel()
    mesh, old = M.keep_vertices(full, wet)
    tri = mesh["tri"]
    H0 = H0_full[old]
    lat_e = mesh["y"][tri].mean(axis=1)
    f = 2.0 * OMEGA * np.sin(lat_e)
    ax = _rms_scale(_elem_mean(ax_full[old], tri), 1.0e-5)
    ay = _rms_scale(_elem_mean(ay_full[old], tri), 1.0e-5)
    He = _elem_mean(H0, tri)
    R = np.stack([He * ax, He * ay], -1)
    eta0 = eta_full[old]
    return _pack(mesh, H0, f, R, eta0, None, tau=960.0, nsub=80, nsteps=nsteps,
                 name=f"C3-latlon-{nlon}x{nlat}")


def vertex_subset(case: dict, vertices: np.ndarray, name: str | None = None):
    """The workload restricted to a set of its vertices (input numbering): the triangles
    with all three vertices in the set, their vertices, and every field on them.  With a
    contiguous range of a space-filling-curve order this is one GPU's share of the mesh
    (its edge becomes a coast instead of a halo)."""
    keep = np.zeros(case["x"].size, bool)
    keep[np.asarray(vertices)] = True
    keep_t = keep[case["tri"]].all(axis=1)
    mesh, old = M.keep_vertices(case, keep)
    d = dict(case)
    d.update(x=mesh["x"], y=mesh["y"], tri=mesh["tri"], H0=case["H0"][old].copy(),
             eta0=case["eta0"][old].copy(), f=case["f"][keep_t].copy(),
             R=case["R"][keep_t].copy(), U0=case["U0"][keep_t].copy(),
             W=None if case.get("W") is None else case["W"][old].copy(),
             name=name or case["name"] + "-subset")
    return d


def adjoint_c5(seed: int = 0, n: int = 256, delta: float = 4000.0):
    """256x256 jittered closed basin with a seeded elevation target."""
    r = M.rng(500 + seed)
    mesh = M.planar_grid(n, n, delta, delta, jitter=0.3, r=r)
    L = (n - 1) * delta
    H0 = 100.0 + 4900.0 * _normalize01(_blobs(mesh["x"], mesh["y"], r, 64, L, L,
                                              40e3, 300e3, False))
    cx, cy = M.element_centroid_planar(mesh)
    ax = _rms_scale(_signed_blobs(cx, cy, r, 64, L, L, 40e3, 300e3, False), 1.0e-5)
    ay = _rms_scale(_signed_blobs(cx, cy, r, 64, L, L, 40e3, 300e3, False), 1.0e-5)
    He = _elem_mean(H0, mesh["tri"])
    R = np.stack([He * ax, He * ay], -1)
    ne = mesh["tri"].shape[0]
    eta0 = _rms_scale(_signed_blobs(mesh["x"], mesh["y"], r, 32, L, L, 60e3, 200e3, False), 0.5)
    target = _rms_scale(_signed_blobs(mesh["x"], mesh["y"], r, 32, L, L, 60e3, 200e3, False), 0.5)
    d = _pack(mesh, H0, np.full(ne, 1.0e-4), R, eta0, None, tau=180.0, nsub=30,
              nsteps=1, name=f"C5-adjoint-{n}x{n}")
    d["eta_target"] = target
    d["ckpt_every"] = 5
    return d


def _member_basin(r, nv_target, aspect, delta, nsub):
    ny = max(8, int(round(np.sqrt(nv_target / aspect))))
    nx = max(8, int(round(nv_target / ny)))
    mesh = M.planar_grid(nx, ny, delta, delta, jitter=0.3, r=r)
    lx, ly = (nx - 1) * delta, (ny - 1) * delta
    zH = _smooth_noise(r, (ny, nx), 12.0, wrap_x=False).ravel()
    H0 = 100.0 + 4900.0 * _normalize01(zH)
    ne = mesh["tri"].shape[0]
    f0 = r.uniform(5.0e-5, 1.4e-4)
    ax_v = _smooth_noise(r, (ny, nx), 16.0, wrap_x=False).ravel()
    ay_v = _smooth_noise(r, (ny, nx), 16.0, wrap_x=False).ravel()
    tri = mesh["tri"]
    ax = _rms_scale(_elem_mean(ax_v, tri), 1.0e-5)
    ay = _rms_scale(_elem_mean(ay_v, tri), 1.0e-5)
    He = _elem_mean(H0, tri)
    R = np.stack([He * ax, He * ay], -1)
    eta0 = _gaussian_eta(mesh, r, 1.0, max(3.0, 0.08 * min(nx, ny)))
    # half of the structured-grid stability limit at the deepest point
    mu_max = 4.0 / delta ** 2 + 4.0 / delta ** 2
    dts = 0.5 * _C_STAB / np.sqrt(G * H0.max() * mu_max)
    return _pack(mesh, H0, np.full(ne, f0), R, eta0, None, tau=nsub * dts, nsub=nsub,
                 nsteps=10, name=f"member-{nx}x{ny}")


def batch_c4(seed: int = 0, nmembers: int = 64, nv_lo: int = 10_000,
             nv_hi: int = 200_000, m_lo: int = 20, m_hi: int = 120):
    """Ensemble of independent jittered basins with uneven sizes and substep counts."""
    r = M.rng(400 + seed)
    members = []
    for _ in range(nmembers):
        nv_t = int(r.integers(nv_lo, nv_hi + 1))
        aspect = r.uniform(1.0, 3.0)
        delta = r.uniform(2.0e3, 20.0e3)
        nsub = int(r.integers(m_lo, m_hi + 1))
        members.append(_member_basin(r, nv_t, aspect, delta, nsub))
    return members


def torus(nx: int, ny: int, dx: float, dy: float, *, H=4000.0, f=0.0, tau=60.0,
          nsub=10, linear_h=True, jitter=0.0, seed=0):
    """Doubly periodic grid with uniform fields (closed-form tests fill them in)."""
    r = M.rng(700 + seed)
    mesh = M.planar_grid(nx, ny, dx, dy, periodic_x=True, periodic_y=True,
                         jitter=jitter, r=r if jitter > 0 else None)
    nv, ne = nx * ny, mesh["tri"].shape[0]
    return _pack(mesh, np.full(nv, H), np.full(ne, f), np.zeros((ne, 2)), np.zeros(nv),
                 None, tau=tau, nsub=nsub, nsteps=1, linear_h=linear_h,
                 name=f"torus-{nx}x{ny}", eta_ref=0.0)


def equilateral_torus(n: int, s: float, *, H=4000.0, tau=60.0, nsub=10):
    """Doubly periodic mesh of equilateral triangles with side s: n x 2n vertices
    (rows sheared by half a side each, so that 2n rows close the torus), uniform
    depth, no rotation or forcing."""
    nx, ny = n, 2 * n
    i, j = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    Px, Py = nx * s, ny * s * np.sqrt(3.0) / 2.0
    x = np.mod(i * s - j * s / 2.0, Px).ravel()
    y = (j * s * np.sqrt(3.0) / 2.0).ravel()
    mesh = dict(x=x, y=y, tri=M.grid_triangles(nx, ny, True, True), periodic_x=True,
                periodic_y=True, period_x=float(Px), period_y=float(Py), spherical=False,
                radius=0.0, nx=nx, ny=ny, dx=s, dy=s * np.sqrt(3.0) / 2.0)
    ne = mesh["tri"].shape[0]
    return _pack(mesh, np.full(nx * ny, H), np.zeros(ne), np.zeros((ne, 2)), np.zeros(nx * ny),
                 None, tau=tau, nsub=nsub, nsteps=1, linear_h=True,
                 name=f"equilateral-torus-{nx}x{ny}", eta_ref=0.0)


def random_case(mesh: dict, seed: int = 0, *, H=(500.0, 4000.0), eta_amp=0.5,
                U_amp=50.0, R_amp=0.05, f=(5e-5, 1.4e-4), tau=24.0, nsub=12,
                linear_h=False):
    """Random (non-smooth) fields on any mesh, for brute-force and derivative tests."""
    r = M.rng(800 + seed)
    nv, ne = mesh["x"].size, mesh["tri"].shape[0]
    H0 = r.uniform(H[0], H[1], nv)
    eta0 = eta_amp * r.standard_normal(nv)
    U0 = U_amp * r.standard_normal((ne, 2))
    R = R_amp * r.standard_normal((ne, 2))
    ff = r.uniform(f[0], f[1], ne)
    return _pack(mesh, H0, ff, R, eta0, U0, tau=tau, nsub=nsub, nsteps=1,
                 linear_h=linear_h, name="random")


def layers(case: dict, K: int = 40, seed: int = 0, *, U_amp: float = 0.5):
    """Synthetic K-layer inputs for the consumer of the averaged transport.

    frac [K]: reference layer fractions of the column (thin at the surface,
    stretched with depth, summing to 1; the shape of a z* grid with 40 levels);
    Ustar [ne][K][2]: layer transports before the trim, a smooth vertical
    profile times random horizontal structure (m^2/s).
    """
    r = M.rng(1300 + seed)
    z = np.arange(K, dtype=np.float64)
    frac = 1.0 + 0.08 * z + 0.002 * z ** 2
    frac = frac / frac.sum()
    ne = case["tri"].shape[0]
    prof = np.cos(np.pi * (z + 0.5) / K)[None, :, None]
    Ustar = U_amp * prof * r.standard_normal((ne, 1, 2)) + 0.1 * U_amp * r.standard_normal((ne, K, 2))
    return dict(frac=frac, Ustar=Ustar, K=K)


def column_forcing(case: dict, K: int = 40, seed: int = 0, *, Cd: float = 2.5e-3):
    """Synthetic baroclinic layer tendencies for the vertically integrated forcing.

    Layer interfaces follow the z* fractions of :func:`layers` over the deepest
    column; an element keeps the layers whose top lies above its depth (mean H0
    of its vertices), so nlev [ne] follows the bathymetry (at least 1).
    RA, RP, RhV [ne][K][2]: advective, pressure (without eta) and horizontal
    viscous transport tendencies, layer thickness times an acceleration of
    order 1e-5, 1e-5 and 1e-6 m/s^2 decaying with depth (m^2/s^2); u [ne][K][2]:
    layer velocities (0.1 m/s scale); tau_s [ne][2]: kinematic surface stress
    (0.1 N/m^2 over 1025 kg/m^3).  Layers at or below nlev hold zeros.
    """
    r = M.rng(1400 + seed)
    frac = layers(case, K=K)["frac"]
    H0 = np.asarray(case["H0"], np.float64)
    He = H0[case["tri"]].mean(axis=1)
    Hmax = H0.max()
    top = Hmax * np.concatenate([[0.0], np.cumsum(frac)[:-1]])
    nlev = np.clip(np.searchsorted(top, He, side="left"), 1, K).astype(np.int32)
    ne = He.size
    h = (Hmax * frac)[None, :, None]
    decay = np.exp(-np.arange(K) / (0.3 * K))[None, :, None]
    mask = (np.arange(K)[None, :] < nlev[:, None])[:, :, None]

    def field(scale, prof):
        a = r.standard_normal((ne, 1, 2)) * prof + 0.3 * r.standard_normal((ne, K, 2))
        return np.where(mask, scale * a, 0.0)

    RA = field(1e-5, decay) * h
    RP = field(1e-5, 1.0 - 0.5 * decay) * h
    RhV = field(1e-6, decay) * h
    u = field(0.1, 0.3 + decay)
    tau_s = 1e-4 * r.standard_normal((ne, 2))
    return dict(K=K, nlev=nlev, RA=RA, RP=RP, RhV=RhV, u=u, tau_s=tau_s, Cd=Cd)


BUILDERS = {"C1": basin_c1, "C2": channel_c2, "C3": latlon_c3, "C4": batch_c4,
            "C5": adjoint_c5}


def make_config(name: str, seed: int = 0, **kw):
    return BUILDERS[name](seed, **kw)
