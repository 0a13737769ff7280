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


def subcycle(ops, eta, U, *, H0, f, R, W=None, g, theta, nsub, tau, linear_h=False):
    """nsub substeps; returns (eta^M, U^M, Uavg) with Uavg per eq. (eq4_12)."""
    dts = tau / nsub
    U0 = np.asarray(U, float).reshape(-1, 2).copy()
    s = np.zeros_like(U0)
    for _ in range(nsub):
        eta, U = substep(ops, eta, U, H0=H0, f=f, R=R, W=W, g=g, theta=theta, dts=dts,
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
