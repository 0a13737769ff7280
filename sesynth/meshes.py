"""Seeded synthetic triangular meshes.

Only input recipes live here (vertex coordinates, triangle connectivity and
the periodicity / sphere flags).  Nothing in this module evaluates any part of
the barotropic scheme; the oracle and the GPU library both consume these
arrays unchanged.

Meshes are returned as a dict:
    x, y        float64 [nv]   metres, or (longitude, latitude) radians if spherical
    tri         int32 [ne, 3]  counter-clockwise vertex triples
    periodic_x, periodic_y     bool
    period_x, period_y         float64 (0 where not periodic)
    spherical   bool
    radius      float64        sphere radius (0 if planar)
    nx, ny      structured-grid shape the mesh was built from (information only)
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20231114
EARTH_RADIUS = 6.371e6


def rng(seed: int) -> np.random.Generator:
    """PCG64 stream for a config; every generator derives from BASE_SEED."""
    return np.random.default_rng(np.random.PCG64(BASE_SEED + int(seed)))


def grid_triangles(nx: int, ny: int, periodic_x: bool = False,
                   periodic_y: bool = False) -> np.ndarray:
    """Triangles of an nx-by-ny vertex grid (vertex id j*nx + i).

    Every quad (i, j)-(i+1, j)-(i+1, j+1)-(i, j+1) is split along the same
    diagonal (i, j)-(i+1, j+1), giving two counter-clockwise triangles.  A
    periodic direction adds the quads that wrap from the last column/row back
    to the first.
    """
    qx = nx if periodic_x else nx - 1
    qy = ny if periodic_y else ny - 1
    ii, jj = np.meshgrid(np.arange(qx, dtype=np.int64), np.arange(qy, dtype=np.int64))
    i1 = (ii + 1) % nx
    j1 = (jj + 1) % ny
    v00 = jj * nx + ii
    v10 = jj * nx + i1
    v11 = j1 * nx + i1
    v01 = j1 * nx + ii
    tri = np.empty((2 * qx * qy, 3), dtype=np.int32)
    tri[0::2] = np.stack([v00, v10, v11], -1).reshape(-1, 3)
    tri[1::2] = np.stack([v00, v11, v01], -1).reshape(-1, 3)
    return tri


def _disc_jitter(r: np.random.Generator, n: int, radius: float):
    """n displacements uniform in a disc of the given radius.

    A disc of radius 0.3 cell keeps every split quad counter-clockwise: each
    vertex moves at most 0.3 cell towards the opposite side, whose distance is
    at least 0.707 cell.
    """
    ang = r.uniform(0.0, 2.0 * np.pi, n)
    rad = radius * np.sqrt(r.uniform(0.0, 1.0, n))
    return rad * np.cos(ang), rad * np.sin(ang)


def planar_grid(nx: int, ny: int, dx: float, dy: float, *, periodic_x=False,
                periodic_y=False, jitter=0.0, r: np.random.Generator | None = None):
    """Structured planar grid, optionally jittered.

    Interior vertices move uniformly inside a disc of radius jitter*min(dx, dy).
    Vertices on a solid wall move only along that wall; corners stay fixed.
    """
    i = np.tile(np.arange(nx, dtype=np.float64), ny)
    j = np.repeat(np.arange(ny, dtype=np.float64), nx)
    x = i * dx
    y = j * dy
    if jitter > 0.0:
        assert r is not None
        jx, jy = _disc_jitter(r, nx * ny, jitter * min(dx, dy))
        on_xwall = np.zeros(nx * ny, bool) if periodic_x else ((i == 0) | (i == nx - 1))
        on_ywall = np.zeros(nx * ny, bool) if periodic_y else ((j == 0) | (j == ny - 1))
        # wall vertices slide along the wall only (1D uniform)
        along = r.uniform(-jitter, jitter, nx * ny)
        jx = np.where(on_ywall, along * dx, jx)
        jy = np.where(on_xwall, along * dy, jy)
        jx = np.where(on_xwall, 0.0, jx)
        jy = np.where(on_ywall, 0.0, jy)
        x = x + jx
        y = y + jy
    mesh = dict(
        x=x, y=y, tri=grid_triangles(nx, ny, periodic_x, periodic_y),
        periodic_x=bool(periodic_x), periodic_y=bool(periodic_y),
        period_x=float(nx * dx) if periodic_x else 0.0,
        period_y=float(ny * dy) if periodic_y else 0.0,
        spherical=False, radius=0.0, nx=nx, ny=ny, dx=dx, dy=dy,
    )
    return mesh


def latlon_grid(nlon: int, nlat: int, lat_min_deg: float, lat_max_deg: float,
                radius: float = EARTH_RADIUS):
    """Longitude-periodic lat-lon grid on a sphere, coordinates in radians."""
    lon = np.arange(nlon, dtype=np.float64) * (2.0 * np.pi / nlon)
    lat = np.deg2rad(np.linspace(lat_min_deg, lat_max_deg, nlat))
    x = np.tile(lon, nlat)
    y = np.repeat(lat, nlon)
    return dict(
        x=x, y=y, tri=grid_triangles(nlon, nlat, periodic_x=True),
        periodic_x=True, periodic_y=False, period_x=2.0 * np.pi, period_y=0.0,
        spherical=True, radius=float(radius), nx=nlon, ny=nlat,
        dx=2.0 * np.pi / nlon, dy=float(lat[1] - lat[0]),
    )


def keep_vertices(mesh: dict, wet: np.ndarray):
    """Drop every triangle touching a dry vertex, then every orphan vertex.

    Returns (new mesh, old index of each kept vertex).  Surviving vertices keep
    their relative order.
    """
    tri = mesh["tri"]
    keep_t = wet[tri].all(axis=1)
    tri = tri[keep_t]
    used = np.zeros(mesh["x"].shape[0], bool)
    used[tri.ravel()] = True
    old = np.nonzero(used)[0]
    new_of_old = -np.ones(mesh["x"].shape[0], np.int64)
    new_of_old[old] = np.arange(old.size)
    out = dict(mesh)
    out["x"] = mesh["x"][old].copy()
    out["y"] = mesh["y"][old].copy()
    out["tri"] = new_of_old[tri].astype(np.int32)
    return out, old


def element_centroid_planar(mesh: dict):
    """Planar centroid of every triangle, unwrapping periodic seams."""
    x, y, tri = mesh["x"], mesh["y"], mesh["tri"]
    cx = []
    cy = []
    for arr, per, out in ((x, mesh["period_x"], cx), (y, mesh["period_y"], cy)):
        p = arr[tri]
        if per > 0.0:
            d = p - p[:, :1]
            d = np.where(d > per / 2, d - per, d)
            d = np.where(d <= -per / 2, d + per, d)
            c = p[:, 0] + d.mean(axis=1)
            c = np.mod(c, per)
        else:
            c = p.mean(axis=1)
        out.append(c)
    return cx[0], cy[0]


def tiny_mesh(kind: str, seed: int = 0):
    """Hand-checkable small meshes for unit tests."""
    r = rng(900 + seed)
    if kind == "two":
        x = np.array([0.0, 1.0, 1.0, 0.0]) * 1000.0
        y = np.array([0.0, 0.0, 1.0, 1.0]) * 1000.0
        tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
        return dict(x=x, y=y, tri=tri, periodic_x=False, periodic_y=False,
                    period_x=0.0, period_y=0.0, spherical=False, radius=0.0,
                    nx=2, ny=2, dx=1000.0, dy=1000.0)
    if kind == "grid3":
        return planar_grid(3, 3, 1000.0, 1000.0)
    if kind == "torus43":
        return planar_grid(4, 3, 1000.0, 1200.0, periodic_x=True, periodic_y=True)
    if kind == "jitter65":
        return planar_grid(6, 5, 1000.0, 1100.0, jitter=0.3, r=r)
    if kind == "jitter76":
        return planar_grid(7, 6, 1500.0, 1300.0, jitter=0.3, r=r)
    if kind == "chan54":
        return planar_grid(5, 4, 1000.0, 900.0, periodic_x=True, jitter=0.3, r=r)
    if kind == "fan100":
        # one vertex shared by 100 triangles (a long CSR row), on a jittered disc
        n = 100
        ang = 2 * np.pi * (np.arange(n) + 0.3 * r.random(n)) / n
        rad = 1000.0 * (1.0 + 0.2 * r.random(n))
        x = np.concatenate([[0.0], rad * np.cos(ang)])
        y = np.concatenate([[0.0], rad * np.sin(ang)])
        i = np.arange(1, n + 1)
        tri = np.stack([np.zeros(n, np.int64), i, i % n + 1], -1).astype(np.int32)
        return dict(x=x, y=y, tri=tri, periodic_x=False, periodic_y=False, period_x=0.0,
                    period_y=0.0, spherical=False, radius=0.0, nx=n + 1, ny=1, dx=60.0, dy=60.0)
    if kind == "sphere86":
        m = latlon_grid(8, 6, -60.0, 60.0, radius=1.0e6)
        return m
    raise ValueError(kind)
