// Host-side mesh preparation: validation, space-filling-curve reordering,
// vertex->triangle CSR, FP64 geometry, spectral bound, and the tile level
// sets of the temporally blocked kernel.  Built with -ffp-contract=off so the
// geometry is the plain IEEE evaluation of its formulas.
#include <algorithm>
#include <atomic>
#include <thread>
#include <cmath>
#include <cstring>
#include <numeric>
#include <tuple>

#include "kernels.h"
#include "se_internal.h"

namespace sesub {

namespace {

// Hilbert index of cell (x, y) on a side x side grid (side a power of two):
// per bit level, quadrant code (3 rx) xor ry, then the sub-square is mapped
// back to the canonical orientation (flip when rx and not ry, transpose when
// not ry).
uint64_t hilbert_index(uint32_t side, uint32_t x, uint32_t y) {
    uint64_t d = 0;
    uint32_t s = side >> 1;
    while (s) {
        const uint32_t rx = (x & s) != 0u, ry = (y & s) != 0u;
        d += static_cast<uint64_t>(s) * s * ((3u * rx) ^ ry);
        if (!ry) {
            if (rx) {
                x = side - 1u - x;
                y = side - 1u - y;
            }
            std::swap(x, y);
        }
        s >>= 1;
    }
    return d;
}

inline uint32_t q16(double v, double lo, double scale) {
    double q = std::floor((v - lo) * scale);
    q = q < 0.0 ? 0.0 : (q > 65535.0 ? 65535.0 : q);
    return static_cast<uint32_t>(q);
}

inline double wrap_period(double d, double per) {
    if (d > 0.5 * per) return d - per;
    if (d <= -0.5 * per) return d + per;
    return d;
}

}  // namespace

se_status build_host_mesh(const se_mesh_desc &d, HostMesh &m) {
    if (!d.x || !d.y || !d.tri || d.nv <= 0 || d.ne <= 0) {
        set_error("se_mesh_create: null array or empty mesh");
        return SE_ERR_ARG;
    }
    if (d.nv >= (int64_t(1) << 31) || d.ne >= (int64_t(1) << 29)) {
        set_error("se_mesh_create: mesh too large for 32-bit indices");
        return SE_ERR_ARG;
    }
    if ((d.flags & SE_SPHERICAL) && !(d.radius > 0.0)) {
        set_error("se_mesh_create: spherical mesh needs radius > 0");
        return SE_ERR_ARG;
    }
    if ((d.flags & SE_PERIODIC_X) && !(d.flags & SE_SPHERICAL) && !(d.period_x > 0.0)) {
        set_error("se_mesh_create: periodic x needs period_x > 0");
        return SE_ERR_ARG;
    }
    if ((d.flags & SE_PERIODIC_Y) && !(d.period_y > 0.0)) {
        set_error("se_mesh_create: periodic y needs period_y > 0");
        return SE_ERR_ARG;
    }
    const int64_t nv = d.nv, ne = d.ne;
    m.nv = nv;
    m.ne = ne;
    m.flags = d.flags;
    m.period_x = d.period_x;
    m.period_y = d.period_y;
    m.radius = d.radius;
    for (int64_t i = 0; i < 3 * ne; ++i) {
        if (d.tri[i] < 0 || d.tri[i] >= nv) {
            set_error("se_mesh_create: triangle vertex index out of range");
            return SE_ERR_MESH;
        }
    }
    for (int64_t i = 0; i < nv; ++i) {
        if (!std::isfinite(d.x[i]) || !std::isfinite(d.y[i])) {
            set_error("se_mesh_create: non-finite coordinate");
            return SE_ERR_MESH;
        }
    }

    // ---- vertices along the Hilbert curve (key, then input index) ----
    double xlo = d.x[0], xhi = d.x[0], ylo = d.y[0], yhi = d.y[0];
    for (int64_t i = 1; i < nv; ++i) {
        xlo = std::min(xlo, d.x[i]);
        xhi = std::max(xhi, d.x[i]);
        ylo = std::min(ylo, d.y[i]);
        yhi = std::max(yhi, d.y[i]);
    }
    const double sx = xhi > xlo ? 65535.0 / (xhi - xlo) : 0.0;
    const double sy = yhi > ylo ? 65535.0 / (yhi - ylo) : 0.0;
    std::vector<uint64_t> vkey(nv);
    for (int64_t i = 0; i < nv; ++i) {
        const uint64_t h = hilbert_index(65536u, q16(d.x[i], xlo, sx), q16(d.y[i], ylo, sy));
        vkey[i] = (h << 32) | static_cast<uint64_t>(i);   // h < 2^32, i < 2^31
    }
    std::sort(vkey.begin(), vkey.end());
    m.vperm.resize(nv);
    std::vector<int32_t> vnew(nv);
    for (int64_t k = 0; k < nv; ++k) {
        const int32_t old = static_cast<int32_t>(vkey[k] & 0xffffffffu);
        m.vperm[k] = old;
        vnew[old] = static_cast<int32_t>(k);
    }

    // ---- triangles: smallest vertex first (cyclic), then lexicographic ----
    struct TK {
        int32_t a, b, c, src;
    };
    std::vector<TK> tk(ne);
    for (int64_t e = 0; e < ne; ++e) {
        int32_t v[3] = {vnew[d.tri[3 * e]], vnew[d.tri[3 * e + 1]], vnew[d.tri[3 * e + 2]]};
        int r = 0;
        if (v[1] < v[r]) r = 1;
        if (v[2] < v[r]) r = 2;
        tk[e] = {v[r], v[(r + 1) % 3], v[(r + 2) % 3], static_cast<int32_t>(e)};
        if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) {
            set_error("se_mesh_create: triangle with a repeated vertex");
            return SE_ERR_MESH;
        }
    }
    std::sort(tk.begin(), tk.end(), [](const TK &p, const TK &q) {
        return std::tie(p.a, p.b, p.c, p.src) < std::tie(q.a, q.b, q.c, q.src);
    });
    m.eperm.resize(ne);
    m.tri.resize(3 * ne);
    for (int64_t e = 0; e < ne; ++e) {
        if (e && tk[e].a == tk[e - 1].a && tk[e].b == tk[e - 1].b && tk[e].c == tk[e - 1].c) {
            set_error("se_mesh_create: duplicate triangle");
            return SE_ERR_MESH;
        }
        m.eperm[e] = tk[e].src;
        m.tri[3 * e] = tk[e].a;
        m.tri[3 * e + 1] = tk[e].b;
        m.tri[3 * e + 2] = tk[e].c;
    }

    // ---- CSR: counting sort, triangles ascending per vertex ----
    m.row_ptr.assign(nv + 1, 0);
    for (int64_t i = 0; i < 3 * ne; ++i) m.row_ptr[m.tri[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) m.row_ptr[v + 1] += m.row_ptr[v];
    m.col.resize(3 * ne);
    {
        std::vector<int32_t> cur(m.row_ptr.begin(), m.row_ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k)
                m.col[cur[m.tri[3 * e + k]]++] = static_cast<int32_t>((e << 2) | k);
    }
    for (int64_t v = 0; v < nv; ++v) {
        if (m.row_ptr[v + 1] == m.row_ptr[v]) {
            set_error("se_mesh_create: vertex not used by any triangle");
            return SE_ERR_MESH;
        }
    }

    // ---- FP64 geometry in the new numbering ----
    m.x.resize(nv);
    m.y.resize(nv);
    for (int64_t k = 0; k < nv; ++k) {
        m.x[k] = d.x[m.vperm[k]];
        m.y[k] = d.y[m.vperm[k]];
    }
    m.Ae.resize(ne);
    m.gN.resize(6 * ne);
    m.Av.assign(nv, 0.0);
    const double two_pi = 2.0 * M_PI;
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t a = m.tri[3 * e], b = m.tri[3 * e + 1], c = m.tri[3 * e + 2];
        double ux = m.x[b] - m.x[a], uy = m.y[b] - m.y[a];
        double vx = m.x[c] - m.x[a], vy = m.y[c] - m.y[a];
        if (d.flags & SE_SPHERICAL) {
            ux = wrap_period(ux, two_pi);
            vx = wrap_period(vx, two_pi);
            const double lat = (m.y[a] + m.y[b] + m.y[c]) / 3.0;
            const double cl = std::cos(lat);
            ux = d.radius * cl * ux;
            vx = d.radius * cl * vx;
            uy = d.radius * uy;
            vy = d.radius * vy;
        } else {
            if (d.flags & SE_PERIODIC_X) {
                ux = wrap_period(ux, d.period_x);
                vx = wrap_period(vx, d.period_x);
            }
            if (d.flags & SE_PERIODIC_Y) {
                uy = wrap_period(uy, d.period_y);
                vy = wrap_period(vy, d.period_y);
            }
        }
        const double det = ux * vy - uy * vx;   // twice the signed area
        if (!(det > 0.0)) {
            set_error("se_mesh_create: triangle with non-positive area (orientation)");
            return SE_ERR_MESH;
        }
        m.Ae[e] = 0.5 * det;
        const double bx = vy / det, by = -vx / det;   // grad of the basis at vertex b
        const double cx = -uy / det, cy = ux / det;   // ... at vertex c
        double *g = &m.gN[6 * e];
        g[0] = -(bx + cx);
        g[1] = -(by + cy);
        g[2] = bx;
        g[3] = by;
        g[4] = cx;
        g[5] = cy;
    }
    // median-dual areas: each triangle gives a third of its area to each vertex,
    // accumulated per vertex in ascending triangle order
    for (int64_t v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int32_t j = m.row_ptr[v]; j < m.row_ptr[v + 1]; ++j) s += m.Ae[m.col[j] >> 2] / 3.0;
        m.Av[v] = s;
    }

    // ---- Gershgorin bound of K = -D G:  K_vu = (1/A_v) sum_e A_e gN_v . gN_u ----
    double mu = 0.0;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t v = 0; v < nv; ++v) {
        row.clear();
        for (int32_t j = m.row_ptr[v]; j < m.row_ptr[v + 1]; ++j) {
            const int64_t e = m.col[j] >> 2;
            const int k = m.col[j] & 3;
            const double *g = &m.gN[6 * e];
            for (int l = 0; l < 3; ++l) {
                const double w = m.Ae[e] * (g[2 * k] * g[2 * l] + g[2 * k + 1] * g[2 * l + 1]);
                const int32_t u = m.tri[3 * e + l];
                bool found = false;
                for (auto &pr : row)
                    if (pr.first == u) {
                        pr.second += w;
                        found = true;
                        break;
                    }
                if (!found) row.emplace_back(u, w);
            }
        }
        double r = 0.0;
        for (auto &pr : row) r += std::fabs(pr.second);
        mu = std::max(mu, r / m.Av[v]);
    }
    m.mu_max = mu;
    return SE_OK;
}

// ---------------------------------------------------------------------------
// Tiles and their K-ring level sets
// ---------------------------------------------------------------------------
// Element neighbours and edge geometry of the barotropic viscous term: for local
// edge j = (t_j, t_{j+1}) of triangle e, the other triangle through that edge (or
// -1 on a coast), found by scanning the CSR row of t_j for a triangle that also
// holds t_{j+1}; the edge length l and l / d, d the distance between the two
// centroids, both placed relative to t_j in the metric of the edge (on the sphere:
// cos of the mean latitude of its two vertices).
se_status build_visc_tables(const HostMesh &m, std::vector<int32_t> &nb4,
                            std::vector<double> &vg) {
    const int64_t ne = m.ne;
    nb4.assign(4 * ne, -1);
    vg.assign(6 * ne, 0.0);
    const bool sph = (m.flags & SE_SPHERICAL) != 0;
    auto rel = [&](int32_t p, int32_t r, double c0, double &dx, double &dy) {
        double ax = m.x[r] - m.x[p], ay = m.y[r] - m.y[p];
        if (sph) {
            ax = wrap_period(ax, 2.0 * M_PI);
            dx = m.radius * c0 * ax;
            dy = m.radius * ay;
        } else {
            if (m.flags & SE_PERIODIC_X) ax = wrap_period(ax, m.period_x);
            if (m.flags & SE_PERIODIC_Y) ay = wrap_period(ay, m.period_y);
            dx = ax;
            dy = ay;
        }
    };
    for (int64_t e = 0; e < ne; ++e) {
        for (int j = 0; j < 3; ++j) {
            const int32_t p = m.tri[3 * e + j], q = m.tri[3 * e + (j + 1) % 3];
            int32_t nb = -1;
            for (int32_t i = m.row_ptr[p]; i < m.row_ptr[p + 1]; ++i) {
                const int32_t t = m.col[i] >> 2;
                if (t == e) continue;
                const int32_t *tt = &m.tri[3 * static_cast<int64_t>(t)];
                if (tt[0] == q || tt[1] == q || tt[2] == q) {
                    if (nb >= 0) {
                        set_error("mesh edge shared by more than two triangles");
                        return SE_ERR_MESH;
                    }
                    nb = t;
                }
            }
            nb4[4 * e + j] = nb;
            if (nb < 0) continue;
            const double c0 = sph ? std::cos(0.5 * (m.y[p] + m.y[q])) : 1.0;
            double ex, ey;
            rel(p, q, c0, ex, ey);
            double cex = 0.0, cey = 0.0, cnx = 0.0, cny = 0.0;
            for (int k = 0; k < 3; ++k) {
                double dx, dy;
                rel(p, m.tri[3 * e + k], c0, dx, dy);
                cex += dx;
                cey += dy;
                rel(p, m.tri[3 * static_cast<int64_t>(nb) + k], c0, dx, dy);
                cnx += dx;
                cny += dy;
            }
            const double ddx = (cnx - cex) / 3.0, ddy = (cny - cey) / 3.0;
            const double l = std::sqrt(ex * ex + ey * ey), d = std::sqrt(ddx * ddx + ddy * ddy);
            if (!(d > 0.0)) {
                set_error("coincident centroids of neighbouring triangles");
                return SE_ERR_MESH;
            }
            vg[6 * e + 2 * j] = l;
            vg[6 * e + 2 * j + 1] = l / d;
        }
    }
    return SE_OK;
}

bool build_trim_tiles(const HostMesh &m, int cap_e, int cap_o, int cap_v, TrimTiles &out) {
    const int64_t nv = m.nv, ne = m.ne;
    out = TrimTiles{};
    out.rloc.assign(3 * static_cast<size_t>(ne), 0);
    std::vector<int32_t> estamp(ne, -1), vstamp(nv, -1), eloc(ne, 0), vloc(nv, 0);
    std::vector<int32_t> te, tv, add_e, add_v;   // this tile's triangles / vertices
    int32_t t = 0;
    for (int64_t v0 = 0; v0 < nv; ++t) {
        te.clear();
        tv.clear();
        int64_t v1 = v0;
        // grow the range while its rows' triangles and their vertices fit
        for (; v1 < nv && v1 - v0 < cap_o; ++v1) {
            add_e.clear();
            add_v.clear();
            for (int32_t j = m.row_ptr[v1]; j < m.row_ptr[v1 + 1]; ++j) {
                const int32_t e = m.col[j] >> 2;
                if (estamp[e] == t) continue;
                estamp[e] = t;
                add_e.push_back(e);
                for (int q = 0; q < 3; ++q) {
                    const int32_t u = m.tri[3 * static_cast<int64_t>(e) + q];
                    if (vstamp[u] != t) {
                        vstamp[u] = t;
                        add_v.push_back(u);
                    }
                }
            }
            if (te.size() + add_e.size() > static_cast<size_t>(cap_e) ||
                tv.size() + add_v.size() > static_cast<size_t>(cap_v)) {
                for (int32_t e : add_e) estamp[e] = -1;
                for (int32_t u : add_v) vstamp[u] = -1;
                break;
            }
            te.insert(te.end(), add_e.begin(), add_e.end());
            tv.insert(tv.end(), add_v.begin(), add_v.end());
        }
        if (v1 == v0) return false;   // one vertex's row alone exceeds the capacity
        // local order: owned triangles (smallest vertex in the range: one contiguous run
        // of the mesh order) then the others, each ascending; owned vertices v0 .. v1 - 1,
        // then the others ascending
        std::sort(te.begin(), te.end());
        std::stable_partition(te.begin(), te.end(), [&](int32_t e) {
            return m.tri[3 * static_cast<int64_t>(e)] >= v0;
        });
        int32_t neo = 0;
        while (neo < static_cast<int32_t>(te.size()) && m.tri[3 * static_cast<int64_t>(te[neo])] >= v0)
            ++neo;
        std::sort(tv.begin(), tv.end());
        const int32_t nvo = static_cast<int32_t>(v1 - v0);
        for (int32_t i = 0; i < nvo; ++i) vloc[v0 + i] = i;
        const int32_t lv_off = static_cast<int32_t>(out.lv.size());
        int32_t nh = 0;
        for (int32_t u : tv)
            if (u < v0 || u >= v1) {
                vloc[u] = nvo + nh++;
                out.lv.push_back(u);
            }
        const int32_t le_off = static_cast<int32_t>(out.le.size() / 2);
        for (int32_t i = 0; i < static_cast<int32_t>(te.size()); ++i) {
            const int32_t e = te[i];
            eloc[e] = i;
            const int32_t *tr = &m.tri[3 * static_cast<int64_t>(e)];
            out.le.push_back(e);
            out.le.push_back(vloc[tr[0]] | vloc[tr[1]] << 10 | vloc[tr[2]] << 20);
        }
        for (int32_t j = m.row_ptr[v0]; j < m.row_ptr[v1]; ++j)
            out.rloc[j] = static_cast<uint16_t>(eloc[m.col[j] >> 2]);
        const int32_t h[8] = {static_cast<int32_t>(v0), nvo, nvo + nh,
                              static_cast<int32_t>(te.size()), neo, lv_off, le_off,
                              m.row_ptr[v1] - m.row_ptr[v0]};
        out.hdr.insert(out.hdr.end(), h, h + 8);
        v0 = v1;
    }
    out.ntiles = t;
    return true;
}

namespace {

// Tiles [t0, t1) of member mi appended to `out` (offsets local to `out`).
se_status build_tile_range(const HostMesh &m, size_t mi, int64_t voff, int64_t eoff,
                           const std::vector<int32_t> &efirst, const std::vector<int32_t> &vstart,
                           int64_t t0, int64_t t1, int32_t K, bool ell,
                           std::vector<int32_t> &vloc, std::vector<int32_t> &eloc,
                           HostTiles &out) {
    std::vector<int32_t> lv, le, fresh, pos;
    for (int64_t t = t0; t < t1; ++t) {
        const int32_t vb = vstart[t];
        const int32_t nv0 = vstart[t + 1] - vb;
        const int32_t eb = efirst[vb], ee = efirst[vb + nv0];
        lv.clear();
        le.clear();
        std::vector<int32_t> nVl(K + 1), nEl(K + 1);
        for (int32_t v = vb; v < vb + nv0; ++v) {
            vloc[v] = static_cast<int32_t>(lv.size());
            lv.push_back(v);
        }
        for (int32_t e = eb; e < ee; ++e) {
            eloc[e] = static_cast<int32_t>(le.size());
            le.push_back(e);
        }
        nVl[0] = nv0;
        nEl[0] = ee - eb;
        for (int32_t i = 1; i <= K; ++i) {
            fresh.clear();
            // triangles touching V_{i-1}: only vertices new at level i-1 can add any
            const int32_t q0 = (i == 1) ? 0 : nVl[i - 2];
            for (int32_t q = q0; q < nVl[i - 1]; ++q) {
                const int32_t v = lv[q];
                for (int32_t j = m.row_ptr[v]; j < m.row_ptr[v + 1]; ++j) {
                    const int32_t e = m.col[j] >> 2;
                    if (eloc[e] == -1) {
                        eloc[e] = -2;   // queued at this level
                        fresh.push_back(e);
                    }
                }
            }
            std::sort(fresh.begin(), fresh.end());
            const size_t e_from = (i == 1) ? 0 : le.size();
            for (int32_t e : fresh) {
                eloc[e] = static_cast<int32_t>(le.size());
                le.push_back(e);
            }
            nEl[i] = static_cast<int32_t>(le.size());
            // new vertices: those of triangles added at this level (all of E_1 at level 1)
            fresh.clear();
            for (size_t q = e_from; q < le.size(); ++q)
                for (int k = 0; k < 3; ++k) {
                    const int32_t v = m.tri[3 * le[q] + k];
                    if (vloc[v] == -1) {
                        vloc[v] = -2;   // queued at this level
                        fresh.push_back(v);
                    }
                }
            std::sort(fresh.begin(), fresh.end());
            for (int32_t v : fresh) {
                vloc[v] = static_cast<int32_t>(lv.size());
                lv.push_back(v);
            }
            nVl[i] = static_cast<int32_t>(lv.size());
        }
        if (nVl[K] > 65535 || 3 * static_cast<int64_t>(nEl[K]) > 65535) {
            for (int32_t v : lv) vloc[v] = -1;
            for (int32_t e : le) eloc[e] = -1;
            set_error("se_set_plan: tile halo too large for 16-bit local indices");
            return SE_ERR_ARG;
        }
        TileHdr h{};
        h.vbase = static_cast<int32_t>(voff + vb);
        h.nv0 = nv0;
        h.ebase = static_cast<int32_t>(eoff + eb);
        h.nown = ee - eb;
        h.lv_off = static_cast<int32_t>(out.lv_gid.size());
        h.le_off = static_cast<int32_t>(out.le_gid.size());
        h.cs_off = 0;
        h.rw_off = static_cast<int32_t>(out.cs_row.size());
        h.member = static_cast<int32_t>(mi);
        h.mtile = static_cast<int32_t>(t);
        // local rows of the vertices updated at some inner substep (V_{K-1}); each
        // incidence (triangle, slot) gets the position where the triangle phase
        // deposits its sub-cell flux: the vertex's row in the local CSR, or with
        // fixed-width rows (ell) entry `rank` of row q at kEllWidth * q + rank, the
        // incidences in ascending triangle order in both.  Incidences of vertices
        // that are never updated go to one of 64 scratch slots past the rows.
        const int32_t nvu = nVl[K - 1];
        pos.assign(3 * le.size(), -1);
        int32_t nent = 0;
        for (int32_t q = 0; q < nvu; ++q) {
            out.cs_row.push_back(static_cast<uint16_t>(nent));
            const int32_t v = lv[q];
            for (int32_t j = m.row_ptr[v]; j < m.row_ptr[v + 1]; ++j) {
                const int32_t e = m.col[j] >> 2;
                const int32_t rank = j - m.row_ptr[v];
                pos[3 * eloc[e] + (m.col[j] & 3)] = ell ? kEllWidth * q + rank : nent;
                ++nent;
            }
        }
        const int32_t rows_end = ell ? kEllWidth * nvu : nent;
        if (rows_end + 64 > 65535) {
            for (int32_t v : lv) vloc[v] = -1;
            for (int32_t e : le) eloc[e] = -1;
            set_error("se_set_plan: tile CSR too large for 16-bit offsets");
            return SE_ERR_ARG;
        }
        out.cs_row.push_back(static_cast<uint16_t>(nent));
        while (out.cs_row.size() % 4) out.cs_row.push_back(0);   // 8-byte vector loads
        out.n_ent += nent;
        out.hdr.push_back(h);
        for (int32_t i = 0; i <= K; ++i) {
            out.nV.push_back(nVl[i]);
            out.nE.push_back(nEl[i]);
        }
        for (int32_t v : lv) out.lv_gid.push_back(static_cast<int32_t>(voff + v));
        for (size_t q = 0; q < le.size(); ++q) {
            const int32_t e = le[q];
            out.le_gid.push_back(static_cast<int32_t>(eoff + e));
            const uint32_t a = vloc[m.tri[3 * e]], b = vloc[m.tri[3 * e + 1]],
                           c = vloc[m.tri[3 * e + 2]];
            uint32_t p3[3];
            for (int k = 0; k < 3; ++k)
                p3[k] = pos[3 * q + k] >= 0 ? static_cast<uint32_t>(pos[3 * q + k])
                                            : static_cast<uint32_t>(rows_end + (q & 63));
            // three local vertices and three flux positions, 16 bits each
            out.le_tri.push_back(a | (b << 16));
            out.le_tri.push_back(c | (p3[0] << 16));
            out.le_tri.push_back(p3[1] | (p3[2] << 16));
        }
        out.max_nv = std::max(out.max_nv, nVl[K]);
        out.max_ne = std::max(out.max_ne, nEl[K]);
        out.max_nvu = std::max(out.max_nvu, nvu);
        out.max_cs = std::max(out.max_cs, rows_end + 64);
        out.max_nown = std::max(out.max_nown, h.nown);
        for (int32_t v : lv) vloc[v] = -1;
        for (int32_t e : le) eloc[e] = -1;
    }
    return SE_OK;
}

}  // namespace

// One pass over the given tile ranges (vstart[mi]: first vertex of each tile of member
// mi, then the member's vertex count), in parallel over runs of tiles.
static se_status build_tiles_pass(const std::vector<const HostMesh *> &members,
                                  const std::vector<int64_t> &voff,
                                  const std::vector<int64_t> &eoff,
                                  const std::vector<std::vector<int32_t>> &vstart,
                                  const std::vector<std::vector<int32_t>> &efirst, int32_t K,
                                  bool ell, HostTiles &out) {
    struct Unit {
        size_t mi;
        int64_t t0, t1;
    };
    std::vector<Unit> units;
    unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    int64_t total_tiles = 0;
    for (size_t mi = 0; mi < members.size(); ++mi) total_tiles += vstart[mi].size() - 1;
    const int64_t chunk = std::max<int64_t>(1, total_tiles / (8 * nthreads));
    for (size_t mi = 0; mi < members.size(); ++mi) {
        const int64_t nt = static_cast<int64_t>(vstart[mi].size()) - 1;
        for (int64_t t = 0; t < nt; t += chunk) units.push_back({mi, t, std::min(nt, t + chunk)});
    }
    std::vector<HostTiles> parts(units.size());
    std::vector<se_status> st(units.size(), SE_OK);
    std::atomic<size_t> next{0};
    auto worker = [&]() {
        std::vector<int32_t> vloc, eloc;
        size_t cur_member = static_cast<size_t>(-1);
        for (;;) {
            const size_t u = next.fetch_add(1);
            if (u >= units.size()) break;
            const Unit &U = units[u];
            const HostMesh &m = *members[U.mi];
            if (U.mi != cur_member) {
                vloc.assign(m.nv, -1);
                eloc.assign(m.ne, -1);
                cur_member = U.mi;
            }
            parts[u].K = K;
            st[u] = build_tile_range(m, U.mi, voff[U.mi], eoff[U.mi], efirst[U.mi],
                                     vstart[U.mi], U.t0, U.t1, K, ell, vloc, eloc, parts[u]);
            if (st[u] != SE_OK) {   // stamps may be dirty after an early return
                cur_member = static_cast<size_t>(-1);
            }
        }
    };
    nthreads = static_cast<unsigned>(std::min<size_t>(nthreads, units.size()));
    std::vector<std::thread> pool;
    for (unsigned k = 1; k < nthreads; ++k) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    for (size_t u = 0; u < units.size(); ++u)
        if (st[u] != SE_OK) {
            set_error("se_set_plan: tile halo or local CSR too large for 16-bit local indices "
                      "(reduce tile or k_fused)");
            return st[u];
        }
    // concatenate in unit order (deterministic), shifting local offsets
    for (size_t u = 0; u < units.size(); ++u) {
        HostTiles &p = parts[u];
        const int32_t dlv = static_cast<int32_t>(out.lv_gid.size());
        const int32_t dle = static_cast<int32_t>(out.le_gid.size());
        const int32_t drw = static_cast<int32_t>(out.cs_row.size());
        for (TileHdr h : p.hdr) {
            h.lv_off += dlv;
            h.le_off += dle;
            h.rw_off += drw;
            out.hdr.push_back(h);
        }
        out.nV.insert(out.nV.end(), p.nV.begin(), p.nV.end());
        out.nE.insert(out.nE.end(), p.nE.begin(), p.nE.end());
        out.lv_gid.insert(out.lv_gid.end(), p.lv_gid.begin(), p.lv_gid.end());
        out.le_gid.insert(out.le_gid.end(), p.le_gid.begin(), p.le_gid.end());
        out.le_tri.insert(out.le_tri.end(), p.le_tri.begin(), p.le_tri.end());
        out.cs_row.insert(out.cs_row.end(), p.cs_row.begin(), p.cs_row.end());
        out.n_ent += p.n_ent;
        out.max_nv = std::max(out.max_nv, p.max_nv);
        out.max_ne = std::max(out.max_ne, p.max_ne);
        out.max_nvu = std::max(out.max_nvu, p.max_nvu);
        out.max_cs = std::max(out.max_cs, p.max_cs);
        out.max_nown = std::max(out.max_nown, p.max_nown);
    }
    return SE_OK;
}

se_status build_tiles(const std::vector<const HostMesh *> &members,
                      const std::vector<int64_t> &voff, const std::vector<int64_t> &eoff,
                      int32_t T, int32_t K, HostTiles &out, int32_t split_cap) {
    out = HostTiles();
    out.T = T;
    out.K = K;
    // fixed-width rows when no vertex of any member has more than kEllWidth triangles
    int32_t max_deg = 0;
    for (const HostMesh *m : members)
        for (int64_t v = 0; v < m->nv; ++v)
            max_deg = std::max(max_deg, m->row_ptr[v + 1] - m->row_ptr[v]);
    out.ell = max_deg <= kEllWidth;
    // first triangle whose smallest vertex is >= v, per member; T vertices per tile
    std::vector<std::vector<int32_t>> efirst(members.size()), vstart(members.size());
    for (size_t mi = 0; mi < members.size(); ++mi) {
        const HostMesh &m = *members[mi];
        std::vector<int32_t> &ef = efirst[mi];
        ef.assign(m.nv + 1, static_cast<int32_t>(m.ne));
        for (int64_t e = m.ne - 1; e >= 0; --e) ef[m.tri[3 * e]] = static_cast<int32_t>(e);
        for (int64_t v = m.nv - 1; v >= 0; --v) ef[v] = std::min(ef[v], ef[v + 1]);
        for (int64_t v = 0; v < m.nv; v += T) vstart[mi].push_back(static_cast<int32_t>(v));
        vstart[mi].push_back(static_cast<int32_t>(m.nv));
    }
    se_status rc = build_tiles_pass(members, voff, eoff, vstart, efirst, K, out.ell, out);
    if (rc != SE_OK) return rc;
    // split_cap > 0: halve every tile with more local triangles than split_cap (its
    // halves again, up to four times), keeping the tiles in vertex order
    for (int round = 0; split_cap > 0 && round < 4 && out.max_ne > split_cap; ++round) {
        std::vector<std::vector<int32_t>> vs(members.size());
        size_t t = 0;
        bool any = false;
        for (size_t mi = 0; mi < members.size(); ++mi) {
            for (size_t i = 0; i + 1 < vstart[mi].size(); ++i, ++t) {
                const int32_t vb = vstart[mi][i], n = vstart[mi][i + 1] - vb;
                vs[mi].push_back(vb);
                if (out.nE[t * (K + 1) + K] > split_cap && n >= 2) {
                    vs[mi].push_back(vb + n / 2);
                    any = true;
                }
            }
            vs[mi].push_back(vstart[mi].back());
        }
        if (!any) break;
        vstart.swap(vs);
        HostTiles next;
        next.T = T;
        next.K = K;
        next.ell = out.ell;
        rc = build_tiles_pass(members, voff, eoff, vstart, efirst, K, next.ell, next);
        if (rc != SE_OK) return rc;
        out = std::move(next);
    }
    return SE_OK;
}

}  // namespace sesub
