"""Brute-force dense stepping from an independent median-dual construction.

TEST INFRASTRUCTURE ONLY.  This module rebuilds the spatial operators of the
barotropic subcycle geometrically, without the closed-form basis gradients
used by ``oracle.c``:

  * gradient: the plane through the three vertex values of each triangle,
    found by solving the 3x3 interpolation system;
  * median-dual cell of a vertex inside a triangle: the quadrilateral
    (vertex, edge midpoint, centroid, edge midpoint); its area by the shoelace
    formula; its outward flux through the two interior segments from the
    segment vectors rotated clockwise (coastline segments carry no flux).

The barotropic viscous term of eq. (eq:viscosity_BT) is rebuilt edge by edge: the
interior edges come from a dictionary of vertex pairs, each edge's two-point flux
is added to one triangle and subtracted from the other, the centroid distance
is a third of the distance between the two vertices opposite the edge, and the
triangle areas come from the shoelace formula.

The substep then follows eq. (eq4_10) of the paper with dense matrices and
numpy.linalg.solve for the Crank-Nicolson Coriolis system (pressure sign of
eq. (eq4_5), see oracle.c); the AB3-AM4 substep of eqs. (eq4_7)-(eq4_8) is
written the same way, with the histories kept as lists of states.
"""
from __future__ import annotations

import numpy as np


def _local_coords(mesh, t):
    """Planar coordinates of the three vertices of one triangle, vertex 0 at origin."""
    x, y = mesh["x"], mesh["y"]
    P = np.zeros((3, 2))
    if mesh.get("spherical"):
        lat_m = np.mean(y[t])
        for k in range(1, 3):
            dl = x[t[k]] - x[t[0]]
            dl = (dl + np.pi) % (2 * np.pi) - np.pi
            if dl == -np.pi:
                dl = np.pi
            P[k] = (mesh["radius"] * np.cos(lat_m) * dl, mesh["radius"] * (y[t[k]] - y[t[0]]))
    else:
        for k in range(1, 3):
            d = np.array([x[t[k]] - x[t[0]], y[t[k]] - y[t[0]]])
            for ax, key in ((0, "period_x"), (1, "period_y")):
                per = mesh.get(key, 0.0)
                if per and per > 0.0:
                    if d[ax] > per / 2:
                        d[ax] -= per
                    elif d[ax] <= -per / 2:
                        d[ax] += per
            P[k] = d
    return P


def _shoelace(poly):
    xs, ys = poly[:, 0], poly[:, 1]
    return 0.5 * np.sum(xs * np.roll(ys, -1) - np.roll(xs, -1) * ys)


def dense_operators(mesh):
    """Dense G [ne*2, nv], D [nv, ne*2], averaging P [ne, nv], Av [nv], Ae [ne]."""
    tri = np.asarray(mesh["tri"])
    nv, ne = mesh["x"].size, tri.shape[0]
    G = np.zeros((2 * ne, nv))
    flux = np.zeros((nv, 2 * ne))   # sum of outward normal vectors per (vertex, triangle)
    P = np.zeros((ne, nv))
    Av = np.zeros(nv)
    Ae = np.zeros(ne)
    for e in range(ne):
        t = tri[e]
        X = _local_coords(mesh, t)
        A3 = np.column_stack([X, np.ones(3)])
        coef = np.linalg.solve(A3, np.eye(3))     # column k: plane of basis function k
        for k in range(3):
            G[2 * e, t[k]] += coef[0, k]
            G[2 * e + 1, t[k]] += coef[1, k]
            P[e, t[k]] += 1.0 / 3.0
        Ae[e] = _shoelace(X)
        C = X.mean(axis=0)
        for k in range(3):
            p, nxt, prv = X[k], X[(k + 1) % 3], X[(k + 2) % 3]
            m1 = 0.5 * (p + nxt)
            m2 = 0.5 * (p + prv)
            cell = np.array([p, m1, C, m2])
            Av[t[k]] += _shoelace(cell)
            nvec = np.zeros(2)
            for a, b in ((m1, C), (C, m2)):        # interior segments, CCW traversal
                d = b - a
                nvec += np.array([d[1], -d[0]])    # outward normal = clockwise rotation
            flux[t[k], 2 * e:2 * e + 2] += nvec
    D = flux / Av[:, None]
    return dict(G=G, D=D, P=P, Av=Av, Ae=Ae, nv=nv, ne=ne)


def substep(ops, eta, U, *, H0, f, R, W=None, g, theta, dts, linear_h=False):
    """One dissipative forward-backward substep with the dense operators."""
    ne = ops["ne"]
    U = np.asarray(U, float).reshape(ne, 2)
    grad = (ops["G"] @ eta).reshape(ne, 2)
    He = ops["P"] @ (H0 if linear_h else H0 + eta)
    a = 0.5 * f * dts
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    Un = np.empty_like(U)
    for e in range(ne):
        lhs = np.eye(2) + a[e] * J
        rhs = (np.eye(2) - a[e] * J) @ U[e] + dts * (-g * He[e] * grad[e] + R[e])
        Un[e] = np.linalg.solve(lhs, rhs)
    F = (1.0 + theta) * Un - theta * U
    div = ops["D"] @ F.reshape(-1)
    eta_n = eta - dts * (div + (0.0 if W is None else W))
    return eta_n, Un


def _edge_vec(mesh, p, r, clat):
    """Vector from vertex p to vertex r in the metric of an edge (cos of its latitude)."""
    x, y = mesh["x"], mesh["y"]
    d = np.array([x[r] - x[p], y[r] - y[p]], dtype=float)
    if mesh.get("spherical"):
        d[0] = (d[0] + np.pi) % (2 * np.pi) - np.pi
        if d[0] == -np.pi:
            d[0] = np.pi
        return np.array([mesh["radius"] * clat * d[0], mesh["radius"] * d[1]])
    for ax, key in ((0, "period_x"), (1, "period_y")):
        per = mesh.get(key, 0.0)
        if per and per > 0.0:
            if d[ax] > per / 2:
                d[ax] -= per
            elif d[ax] <= -per / 2:
                d[ax] += per
    return d


def interior_edges(mesh):
    """[(e1, e2, p, q)] for every edge shared by two triangles (p, q its vertices)."""
    tri = np.asarray(mesh["tri"])
    pairs = {}
    for e in range(tri.shape[0]):
        for j in range(3):
            p, q = int(tri[e, j]), int(tri[e, (j + 1) % 3])
            pairs.setdefault((min(p, q), max(p, q)), []).append(e)
    out = []
    for (p, q), es in pairs.items():
        assert len(es) <= 2, "edge shared by more than two triangles"
        if len(es) == 2:
            out.append((es[0], es[1], p, q))
    return out


def visc_operator(mesh, eta, U, *, H0, A0, Cv, linear_h=False, return_energy=False):
    """R^hV = div(H A grad(U/H)) per triangle: two-point fluxes H_j A_j (l/d) (u_2 - u_1)
    through interior edges, A_j = A0 + Cv l |u_2 - u_1|, H_j the mean depth at the edge's
    vertices, u = U / H_e (H_e the triangle mean depth).  With return_energy, also
    -sum over edges of H_j A_j (l/d) |u_2 - u_1|^2."""
    tri = np.asarray(mesh["tri"])
    ne = tri.shape[0]
    U = np.asarray(U, float).reshape(ne, 2)
    Hv = H0 if linear_h else H0 + eta
    He = Hv[tri].mean(axis=1)
    u = U / He[:, None]
    Ae = np.array([_shoelace(_local_coords(mesh, tri[e])) for e in range(ne)])
    V = np.zeros((ne, 2))
    energy = 0.0
    y = mesh["y"]
    for e1, e2, p, q in interior_edges(mesh):
        clat = np.cos(0.5 * (y[p] + y[q])) if mesh.get("spherical") else 1.0
        r1 = [v for v in tri[e1] if v not in (p, q)][0]
        r2 = [v for v in tri[e2] if v not in (p, q)][0]
        l = np.linalg.norm(_edge_vec(mesh, p, q, clat))
        d = np.linalg.norm(_edge_vec(mesh, p, r2, clat) - _edge_vec(mesh, p, r1, clat)) / 3.0
        du = u[e2] - u[e1]
        A = A0 + Cv * l * np.linalg.norm(du)
        F = 0.5 * (Hv[p] + Hv[q]) * A * (l / d) * du
        V[e1] += F / Ae[e1]
        V[e2] -= F / Ae[e2]
        energy -= 0.5 * (Hv[p] + Hv[q]) * A * (l / d) * (du @ du)
    return (V, energy) if return_energy else V


def subcycle(ops, eta, U, *, H0, f, R, W=None, g, theta, nsub, tau, linear_h=False,
             visc=None, mesh=None):
    """nsub substeps; returns (eta^M, U^M, Uavg) with Uavg per eq. (eq4_12).  visc =
    (A0, Cv) with the mesh adds the viscous term at each substep and subtracts its
    value at the start from R."""
    dts = tau / nsub
    U0 = np.asarray(U, float).reshape(-1, 2).copy()
    s = np.zeros_like(U0)
    if visc is not None:
        Rb = R - visc_operator(mesh, eta, U0, H0=H0, A0=visc[0], Cv=visc[1], linear_h=linear_h)
    for _ in range(nsub):
        Rm = R if visc is None else Rb + visc_operator(mesh, eta, U, H0=H0, A0=visc[0],
                                                       Cv=visc[1], linear_h=linear_h)
        eta, U = substep(ops, eta, U, H0=H0, f=f, R=Rm, W=W, g=g, theta=theta, dts=dts,
                         linear_h=linear_h)
        s += U
    Uavg = s / nsub + theta / nsub * (U - U0)
    return eta, U, Uavg


def linear_step_matrix(ops, *, H, theta, dts):
    """Matrix of one substep on (eta, U) for f = 0, R = 0, H = H (linear, uniform)."""
    nv, ne = ops["nv"], ops["ne"]
    n = nv + 2 * ne
    Mx = np.zeros((n, n))
    for j in range(n):
        z = np.zeros(n)
        z[j] = 1.0
        eta, U = z[:nv], z[nv:].reshape(ne, 2)
        en, Un = substep(ops, eta, U, H0=np.full(nv, H), f=np.zeros(ne),
                         R=np.zeros((ne, 2)), g=9.81, theta=theta, dts=dts, linear_h=True)
        Mx[:nv, j] = en
        Mx[nv:, j] = Un.reshape(-1)
    return Mx


def subcycle_sesm(ops, eta, U, *, H0, f, R, W=None, g, beta, delta, gamma, zeta, nsub, tau,
                  linear_h=False):
    """AB3-AM4 subcycle with the dense operators; histories start from the initial
    state.  Returns (eta^M, U^M, mean of the AB3 transports)."""
    dts = tau / nsub
    ne = ops["ne"]
    Us = [np.asarray(U, float).reshape(ne, 2).copy()] * 3      # U^m, U^{m-1}, U^{m-2}
    etas = [np.asarray(eta, float).copy()] * 3
    ab = np.array([1.5 + beta, -(0.5 + 2.0 * beta), beta])
    am = np.array([delta, 1.0 - delta - gamma - zeta, gamma, zeta])
    fz = np.asarray(f, float)[:, None]
    acc = np.zeros((ne, 2))
    for _ in range(nsub):
        Uab = ab[0] * Us[0] + ab[1] * Us[1] + ab[2] * Us[2]
        eta_n = etas[0] - dts * (ops["D"] @ Uab.reshape(-1) + (0.0 if W is None else W))
        eam = am[0] * eta_n + am[1] * etas[0] + am[2] * etas[1] + am[3] * etas[2]
        grad = (ops["G"] @ eam).reshape(ne, 2)
        He = ops["P"] @ (H0 if linear_h else H0 + eam)
        cor = np.column_stack([fz[:, 0] * Uab[:, 1], -fz[:, 0] * Uab[:, 0]])   # -f e_z x U
        Un = Us[0] + dts * (cor - g * He[:, None] * grad + np.asarray(R, float).reshape(ne, 2))
        Us = [Un, Us[0], Us[1]]
        etas = [eta_n, etas[0], etas[1]]
        acc += Uab
    return etas[0], Us[0], acc / nsub
