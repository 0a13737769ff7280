/*
 * Plain FP64 CPU oracle of the split-explicit barotropic subcycle
 * (Banerjee et al., "Split-explicit external mode solver in finite volume sea
 * ice ocean model FESOM2", arXiv 2311.08241).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this file's library.  It shares no code
 * with the GPU library and must stay slow, plain and obviously correct:
 * loops in the order of the definitions, no blocking, no fusion.
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC (OpenMP
 * only in orc_subcycle_threads, the all-core timing form of the subcycle).
 *
 * What is computed (readings of the paper fixed where it is silent):
 *  - Continuous problem: the barotropic system of Sec. 2.2, eq. (eq4_5):
 *      dU/dt + f e_z x U + g H grad(eta) = R,  d(eta)/dt + div U + W = 0,
 *    H = H0 + eta, R frozen over the baroclinic step.
 *  - Time stepping: the dissipative forward-backward substep of eq. (eq4_10):
 *    U first with Crank-Nicolson Coriolis, then eta from the divergence of
 *    (1+theta) U^{m+1} - theta U^m.  The printed "- g H grad(eta)" inside the
 *    bracket with a leading minus would flip the pressure force against
 *    eq. (eq4_5) and eq. (eq4_8); the sign of eq. (eq4_5) is used.  W is kept
 *    in the eta line as in eq. (eq4_5).
 *  - Space: scalars at vertices, transports on triangles (Sec. 2.1).  The
 *    gradient is the P1 gradient on each triangle; the divergence is the
 *    median-dual finite-volume divergence (edge midpoints joined to the
 *    centroid), with no flux through coastlines.
 *  - H at substep m is the triangle mean of H0 + eta^m (vertex values).
 *  - Averaged transport: eq. (eq4_12), with the sum over m = 1..M and the
 *    endpoint term theta/M (U^M - U^0), the only reading that makes the summed
 *    elevation equation eq. (eq4_11) exact.
 *  - Alternatives and companions of the subcycle, each documented at its
 *    function: the AB3-AM4 substep of eqs. (eq4_7)-(eq4_8); the barotropic
 *    viscous regularization of eq. (eq:viscosity_BT) with its initial value
 *    subtracted from R; the vertically integrated baroclinic forcing of
 *    eq. (eq4_4); the trim of layer transports (eq. (eq4_13)) with z*
 *    thicknesses and the diasurface velocity (Sec. 2.4).
 *  - Space-filling-curve reordering (not part of the paper's method): a
 *    Hilbert index on a 2^16 x 2^16 quantisation of the coordinates, used to
 *    check the GPU library's reordering integer for integer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PERIODIC_X 1u
#define ORC_PERIODIC_Y 2u
#define ORC_SPHERICAL 4u

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MESH 2
#define ORC_ERR_OOM 3

/* ------------------------------------------------------------------------ */
/* Hilbert curve index (Hilbert 1891; the iterative xy -> d formulation with
 * quadrant code (3 rx) xor ry and a flip/transpose when ry == 0).            */
/* ------------------------------------------------------------------------ */
uint64_t orc_hilbert_d(uint32_t side, uint32_t x, uint32_t y)
{
    uint64_t d = 0;
    for (uint32_t s = side / 2; s > 0; s /= 2) {
        uint32_t rx = (x & s) ? 1u : 0u;
        uint32_t ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * (uint64_t)s * (uint64_t)((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = side - 1 - x;
                y = side - 1 - y;
            }
            uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

/* Quantise one coordinate onto 0..65535 (scale 65535/range, floor, cap). */
static uint32_t quantise(double v, double vmin, double scale)
{
    double q = floor((v - vmin) * scale);
    if (q < 0.0) q = 0.0;
    if (q > 65535.0) q = 65535.0;
    return (uint32_t)q;
}

int orc_sfc_keys(int64_t nv, const double *x, const double *y, uint32_t *key)
{
    if (nv <= 0) return ORC_ERR_ARG;
    double xmin = x[0], xmax = x[0], ymin = y[0], ymax = y[0];
    for (int64_t i = 1; i < nv; ++i) {
        if (x[i] < xmin) xmin = x[i];
        if (x[i] > xmax) xmax = x[i];
        if (y[i] < ymin) ymin = y[i];
        if (y[i] > ymax) ymax = y[i];
    }
    double sx = (xmax > xmin) ? 65535.0 / (xmax - xmin) : 0.0;
    double sy = (ymax > ymin) ? 65535.0 / (ymax - ymin) : 0.0;
    for (int64_t i = 0; i < nv; ++i)
        key[i] = (uint32_t)orc_hilbert_d(65536u, quantise(x[i], xmin, sx), quantise(y[i], ymin, sy));
    return ORC_OK;
}

typedef struct { uint32_t key; int32_t idx; } vkey_t;
typedef struct { int32_t v[3]; int32_t idx; } tkey_t;

static int cmp_vkey(const void *a, const void *b)
{
    const vkey_t *p = (const vkey_t *)a, *q = (const vkey_t *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

static int cmp_tkey(const void *a, const void *b)
{
    const tkey_t *p = (const tkey_t *)a, *q = (const tkey_t *)b;
    for (int k = 0; k < 3; ++k)
        if (p->v[k] != q->v[k]) return p->v[k] < q->v[k] ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

/*
 * Reorder a mesh:
 *  vperm[new] = old vertex (stable sort by Hilbert key, ties by old index);
 *  each triangle renumbered and rotated cyclically so its smallest vertex is
 *  first (orientation kept); eperm[new] = old triangle (lexicographic sort of
 *  the rotated triples; a repeated triple is a mesh error);
 *  row_ptr/col: per vertex, its incident triangles in ascending new index,
 *  encoded (e << 2) | local slot.
 */
int orc_reorder(int64_t nv, int64_t ne, const double *x, const double *y,
                const int32_t *tri, int32_t *vperm, int32_t *eperm,
                int32_t *tri_new, int32_t *row_ptr, int32_t *col)
{
    if (nv <= 0 || ne <= 0) return ORC_ERR_ARG;
    for (int64_t i = 0; i < 3 * ne; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return ORC_ERR_MESH;
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * nv);
    vkey_t *vk = (vkey_t *)malloc(sizeof(vkey_t) * nv);
    int32_t *vinv = (int32_t *)malloc(sizeof(int32_t) * nv);
    tkey_t *tk = (tkey_t *)malloc(sizeof(tkey_t) * ne);
    if (!key || !vk || !vinv || !tk) {
        free(key); free(vk); free(vinv); free(tk);
        return ORC_ERR_OOM;
    }
    orc_sfc_keys(nv, x, y, key);
    for (int64_t i = 0; i < nv; ++i) { vk[i].key = key[i]; vk[i].idx = (int32_t)i; }
    qsort(vk, (size_t)nv, sizeof(vkey_t), cmp_vkey);
    for (int64_t i = 0; i < nv; ++i) { vperm[i] = vk[i].idx; vinv[vk[i].idx] = (int32_t)i; }

    for (int64_t e = 0; e < ne; ++e) {
        int32_t a = vinv[tri[3 * e]], b = vinv[tri[3 * e + 1]], c = vinv[tri[3 * e + 2]];
        int32_t r0, r1, r2;
        if (a <= b && a <= c) { r0 = a; r1 = b; r2 = c; }
        else if (b <= a && b <= c) { r0 = b; r1 = c; r2 = a; }
        else { r0 = c; r1 = a; r2 = b; }
        tk[e].v[0] = r0; tk[e].v[1] = r1; tk[e].v[2] = r2; tk[e].idx = (int32_t)e;
    }
    qsort(tk, (size_t)ne, sizeof(tkey_t), cmp_tkey);
    int status = ORC_OK;
    for (int64_t e = 0; e < ne; ++e) {
        if (e > 0 && tk[e].v[0] == tk[e - 1].v[0] && tk[e].v[1] == tk[e - 1].v[1] &&
            tk[e].v[2] == tk[e - 1].v[2]) status = ORC_ERR_MESH;
        if (tk[e].v[0] == tk[e].v[1] || tk[e].v[1] == tk[e].v[2] || tk[e].v[0] == tk[e].v[2])
            status = ORC_ERR_MESH;
        eperm[e] = tk[e].idx;
        for (int k = 0; k < 3; ++k) tri_new[3 * e + k] = tk[e].v[k];
    }
    /* CSR by counting; triangles visited in ascending new index */
    for (int64_t v = 0; v <= nv; ++v) row_ptr[v] = 0;
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) row_ptr[tri_new[3 * e + k] + 1] += 1;
    for (int64_t v = 0; v < nv; ++v) row_ptr[v + 1] += row_ptr[v];
    int32_t *fill = vinv; /* reuse as cursor */
    for (int64_t v = 0; v < nv; ++v) fill[v] = row_ptr[v];
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int32_t v = tri_new[3 * e + k];
            col[fill[v]++] = (int32_t)((e << 2) | k);
        }
    free(key); free(vk); free(vinv); free(tk);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */
static double wrap_half(double d, double period)
{
    /* into (-period/2, period/2] */
    if (d > 0.5 * period) d -= period;
    else if (d <= -0.5 * period) d += period;
    return d;
}

/*
 * Per triangle e = (a, b, c): area A_e and P1 basis gradients gN[e][k][2]
 * (k = local slot).  Per vertex: median-dual area A_v = sum_e A_e / 3.
 * Planar coordinates: differences wrapped across periodic seams.
 * Spherical coordinates (lon, lat in radians): dx = R cos(mean lat) dlon,
 * dy = R dlat, with dlon wrapped into (-pi, pi].
 */
int orc_geometry(int64_t nv, int64_t ne, const double *x, const double *y,
                 const int32_t *tri, uint32_t flags, double period_x, double period_y,
                 double radius, double *Ae, double *gN, double *Av)
{
    for (int64_t v = 0; v < nv; ++v) Av[v] = 0.0;
    for (int64_t e = 0; e < ne; ++e) {
        int32_t a = tri[3 * e], b = tri[3 * e + 1], c = tri[3 * e + 2];
        double abx = x[b] - x[a], aby = y[b] - y[a];
        double acx = x[c] - x[a], acy = y[c] - y[a];
        if (flags & ORC_SPHERICAL) {
            double pi = 3.14159265358979323846;
            abx = wrap_half(abx, 2.0 * pi);
            acx = wrap_half(acx, 2.0 * pi);
            double latm = (y[a] + y[b] + y[c]) / 3.0;
            double cl = cos(latm);
            abx = radius * cl * abx;
            acx = radius * cl * acx;
            aby = radius * aby;
            acy = radius * acy;
        } else {
            if (flags & ORC_PERIODIC_X) { abx = wrap_half(abx, period_x); acx = wrap_half(acx, period_x); }
            if (flags & ORC_PERIODIC_Y) { aby = wrap_half(aby, period_y); acy = wrap_half(acy, period_y); }
        }
        double twoA = abx * acy - aby * acx;
        if (!(twoA > 0.0)) return ORC_ERR_MESH;
        Ae[e] = 0.5 * twoA;
        double gbx = acy / twoA, gby = -acx / twoA;
        double gcx = -aby / twoA, gcy = abx / twoA;
        gN[6 * e + 0] = -(gbx + gcx);
        gN[6 * e + 1] = -(gby + gcy);
        gN[6 * e + 2] = gbx;
        gN[6 * e + 3] = gby;
        gN[6 * e + 4] = gcx;
        gN[6 * e + 5] = gcy;
        Av[a] += Ae[e] / 3.0;
        Av[b] += Ae[e] / 3.0;
        Av[c] += Ae[e] / 3.0;
    }
    for (int64_t v = 0; v < nv; ++v)
        if (!(Av[v] > 0.0)) return ORC_ERR_MESH;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Forward substep                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t nv, ne;
    const int32_t *tri;
    const double *Ae, *gN, *Av;
} orc_mesh;

/* Triangle-local quantities of one substep, kept so that the derivative code
 * can reuse them without re-deriving anything. */
typedef struct {
    double gx, gy;   /* P1 gradient of eta on the triangle           */
    double He;       /* mean of H0 + eta (or of H0) over the vertices */
    double al;       /* f dt_s / 2                                   */
} orc_elem;

static void elem_quantities(const orc_mesh *m, int64_t e, const double *eta,
                            const double *H0, double f, double dts, int linear_h,
                            orc_elem *q)
{
    const int32_t *t = m->tri + 3 * e;
    const double *g = m->gN + 6 * e;
    /* difference form: constant eta has an exactly zero gradient */
    double db = eta[t[1]] - eta[t[0]], dc = eta[t[2]] - eta[t[0]];
    q->gx = db * g[2] + dc * g[4];
    q->gy = db * g[3] + dc * g[5];
    if (linear_h)
        q->He = (H0[t[0]] + H0[t[1]] + H0[t[2]]) / 3.0;
    else
        q->He = ((H0[t[0]] + eta[t[0]]) + (H0[t[1]] + eta[t[1]]) + (H0[t[2]] + eta[t[2]])) / 3.0;
    q->al = 0.5 * f * dts;
}

/* Ub' = (I + al J)^-1 [ (I - al J) Ub + dts (-g He grad eta + R) ],  J(x,y) = (-y,x) */
static void transport_update(const orc_elem *q, double g, double dts, const double *U,
                             const double *R, double *Un)
{
    double rx = U[0] + q->al * U[1] + dts * (-g * q->He * q->gx + R[0]);
    double ry = U[1] - q->al * U[0] + dts * (-g * q->He * q->gy + R[1]);
    double den = 1.0 + q->al * q->al;
    Un[0] = (rx + q->al * ry) / den;
    Un[1] = (ry - q->al * rx) / den;
}

/* outward flux of F through the sub-cell boundary of slot k inside triangle e:
 * F . S_{e,k}, S_{e,k} = -A_e gN_{e,k} */
static double slot_flux(const orc_mesh *m, int64_t e, int k, const double *F)
{
    const double *g = m->gN + 6 * e + 2 * k;
    double Sx = -m->Ae[e] * g[0], Sy = -m->Ae[e] * g[1];
    return F[0] * Sx + F[1] * Sy;
}

static double volume_of(const orc_mesh *m, const double *eta)
{
    double V = 0.0;
    for (int64_t v = 0; v < m->nv; ++v) V += m->Av[v] * eta[v];
    return V;
}

/*
 * One baroclinic step: nsub substeps of length tau/nsub from (eta, U) in place.
 * Uavg [ne][2] receives the averaged transport, volume [nsub+1] (optional)
 * the volume sum_v A_v eta_v after each substep (entry 0: initial state).
 */
/* Barotropic viscous regularization (eq. (eq:viscosity_BT)) on the element
 * neighbours of each triangle; see orc_visc_apply below. */
typedef struct {
    const int32_t *nb;
    const double *elen, *lod;
    double A0, Cv;
} orc_visc;

static void visc_apply(const orc_mesh *m, const orc_visc *vs, int linear_h, const double *H0,
                       const double *eta, const double *U, double *V);

static int subcycle_core(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                         const double *gN, const double *Av, double g, double theta,
                         int linear_h, const double *H0, const double *f, const double *R,
                         const double *W, int32_t nsub, double tau, double *eta, double *U,
                         double *Uavg, double *volume, const orc_visc *vs)
{
    if (nsub <= 0 || nv <= 0 || ne <= 0) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, gN, Av};
    double dts = tau / (double)nsub;
    double *Un = (double *)malloc(sizeof(double) * 2 * ne);
    double *F = (double *)malloc(sizeof(double) * 2 * ne);
    double *U0 = (double *)malloc(sizeof(double) * 2 * ne);
    double *sum = (double *)calloc((size_t)(2 * ne), sizeof(double));
    double *div = (double *)malloc(sizeof(double) * nv);
    /* with viscosity: Rb = R - V(eta^0, U^0) once, Rm = Rb + V(eta^m, U^m) per substep */
    double *Rb = vs ? (double *)malloc(sizeof(double) * 2 * ne) : NULL;
    double *Rm = vs ? (double *)malloc(sizeof(double) * 2 * ne) : NULL;
    if (!Un || !F || !U0 || !sum || !div || (vs && (!Rb || !Rm))) {
        free(Un); free(F); free(U0); free(sum); free(div); free(Rb); free(Rm);
        return ORC_ERR_OOM;
    }
    memcpy(U0, U, sizeof(double) * 2 * ne);
    if (vs) {
        visc_apply(&m, vs, linear_h, H0, eta, U, Rb);
        for (int64_t i = 0; i < 2 * ne; ++i) Rb[i] = R[i] - Rb[i];
    }
    if (volume) volume[0] = volume_of(&m, eta);
    for (int32_t s = 0; s < nsub; ++s) {
        const double *Rs = R;
        if (vs) {
            visc_apply(&m, vs, linear_h, H0, eta, U, Rm);
            for (int64_t i = 0; i < 2 * ne; ++i) Rm[i] = Rb[i] + Rm[i];
            Rs = Rm;
        }
        for (int64_t e = 0; e < ne; ++e) {
            orc_elem q;
            elem_quantities(&m, e, eta, H0, f[e], dts, linear_h, &q);
            transport_update(&q, g, dts, U + 2 * e, Rs + 2 * e, Un + 2 * e);
            F[2 * e] = (1.0 + theta) * Un[2 * e] - theta * U[2 * e];
            F[2 * e + 1] = (1.0 + theta) * Un[2 * e + 1] - theta * U[2 * e + 1];
        }
        for (int64_t v = 0; v < nv; ++v) div[v] = 0.0;
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k) div[tri[3 * e + k]] += slot_flux(&m, e, k, F + 2 * e);
        for (int64_t v = 0; v < nv; ++v)
            eta[v] = eta[v] - dts * (div[v] / Av[v] + (W ? W[v] : 0.0));
        for (int64_t i = 0; i < 2 * ne; ++i) {
            U[i] = Un[i];
            sum[i] += Un[i];
        }
        if (volume) volume[s + 1] = volume_of(&m, eta);
    }
    for (int64_t i = 0; i < 2 * ne; ++i)
        Uavg[i] = sum[i] / (double)nsub + theta / (double)nsub * (U[i] - U0[i]);
    free(Un); free(F); free(U0); free(sum); free(div); free(Rb); free(Rm);
    return ORC_OK;
}

int orc_subcycle(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                 const double *gN, const double *Av, double g, double theta,
                 int linear_h, const double *H0, const double *f, const double *R,
                 const double *W, int32_t nsub, double tau, double *eta, double *U,
                 double *Uavg, double *volume)
{
    return subcycle_core(nv, ne, tri, Ae, gN, Av, g, theta, linear_h, H0, f, R, W, nsub, tau,
                         eta, U, Uavg, volume, NULL);
}

/* The subcycle with the barotropic viscous regularization of eq. (eq:viscosity_BT)
 * added to the transport equation, evaluated explicitly at substep m, and its
 * value at the start of the subcycle subtracted from R (Sec. 2.2, after eq. (eq4_5)). */
int orc_subcycle_visc(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                      const double *gN, const double *Av, double g, double theta,
                      int linear_h, const double *H0, const double *f, const double *R,
                      const double *W, int32_t nsub, double tau, double *eta, double *U,
                      double *Uavg, double *volume, const int32_t *nb, const double *elen,
                      const double *lod, double A0, double Cv)
{
    if (!nb || !elen || !lod || !(A0 >= 0.0) || !(Cv >= 0.0)) return ORC_ERR_ARG;
    orc_visc vs = {nb, elen, lod, A0, Cv};
    return subcycle_core(nv, ne, tri, Ae, gN, Av, g, theta, linear_h, H0, f, R, W, nsub, tau,
                         eta, U, Uavg, volume, &vs);
}

/*
 * The subcycle of orc_subcycle on several host threads (OpenMP), for timing the
 * definition on all cores of a machine.  Same operations, same order per output:
 *  - the triangle loop computes U', F and the three sub-cell fluxes of each
 *    triangle exactly as above, storing the fluxes instead of adding them;
 *  - each vertex then adds its fluxes starting from 0.0 in ascending triangle
 *    index (its incidences listed by a counting pass over the triangles), which
 *    is the sequence of additions the triangle-order scatter above makes into
 *    that vertex's sum;
 * so eta, U and Uavg equal orc_subcycle's bit for bit for any thread count.  The
 * volume is summed in fixed blocks of 8192 vertices, the block sums then added in
 * block order: independent of the thread count, equal to the serial sum up to
 * rounding.  nthreads <= 0 takes the OpenMP default; *used receives the count.
 * No viscous term.
 */
int orc_subcycle_threads(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                         const double *gN, const double *Av, double g, double theta,
                         int linear_h, const double *H0, const double *f, const double *R,
                         const double *W, int32_t nsub, double tau, double *eta, double *U,
                         double *Uavg, double *volume, int nthreads, int *used)
{
    if (nsub <= 0 || nv <= 0 || ne <= 0) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, gN, Av};
    const double dts = tau / (double)nsub;
    const int64_t VB = 8192, nb = (nv + VB - 1) / VB;
    double *Un = (double *)malloc(sizeof(double) * 2 * ne);
    double *U0 = (double *)malloc(sizeof(double) * 2 * ne);
    double *sum = (double *)calloc((size_t)(2 * ne), sizeof(double));
    double *phi = (double *)malloc(sizeof(double) * 3 * ne);
    double *part = (double *)malloc(sizeof(double) * nb);
    int64_t *row = (int64_t *)calloc((size_t)(nv + 1), sizeof(int64_t));
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * 3 * ne);
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * nv);
    if (!Un || !U0 || !sum || !phi || !part || !row || !slot || !cur) {
        free(Un); free(U0); free(sum); free(phi); free(part); free(row); free(slot); free(cur);
        return ORC_ERR_OOM;
    }
    for (int64_t i = 0; i < 3 * ne; ++i) {
        if (tri[i] < 0 || tri[i] >= nv) {
            free(Un); free(U0); free(sum); free(phi); free(part); free(row); free(slot); free(cur);
            return ORC_ERR_MESH;
        }
        row[tri[i] + 1] += 1;
    }
    for (int64_t v = 0; v < nv; ++v) row[v + 1] += row[v];
    for (int64_t v = 0; v < nv; ++v) cur[v] = row[v];
    for (int64_t i = 0; i < 3 * ne; ++i) slot[cur[tri[i]]++] = i;   /* 3 e + k, e ascending */
    memcpy(U0, U, sizeof(double) * 2 * ne);
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    if (used) *used = nt;
#pragma omp parallel num_threads(nt)
    {
        for (int32_t s = -1; s < nsub; ++s) {
            if (s >= 0) {
#pragma omp for schedule(static)
                for (int64_t e = 0; e < ne; ++e) {
                    orc_elem q;
                    double F[2];
                    elem_quantities(&m, e, eta, H0, f[e], dts, linear_h, &q);
                    transport_update(&q, g, dts, U + 2 * e, R + 2 * e, Un + 2 * e);
                    F[0] = (1.0 + theta) * Un[2 * e] - theta * U[2 * e];
                    F[1] = (1.0 + theta) * Un[2 * e + 1] - theta * U[2 * e + 1];
                    for (int k = 0; k < 3; ++k) phi[3 * e + k] = slot_flux(&m, e, k, F);
                }
#pragma omp for schedule(static)
                for (int64_t v = 0; v < nv; ++v) {
                    double div = 0.0;
                    for (int64_t j = row[v]; j < row[v + 1]; ++j) div += phi[slot[j]];
                    eta[v] = eta[v] - dts * (div / Av[v] + (W ? W[v] : 0.0));
                }
#pragma omp for schedule(static)
                for (int64_t i = 0; i < 2 * ne; ++i) {
                    U[i] = Un[i];
                    sum[i] += Un[i];
                }
            }
            if (volume) {
#pragma omp for schedule(static)
                for (int64_t b = 0; b < nb; ++b) {
                    double V = 0.0;
                    const int64_t v1 = (b + 1) * VB < nv ? (b + 1) * VB : nv;
                    for (int64_t v = b * VB; v < v1; ++v) V += Av[v] * eta[v];
                    part[b] = V;
                }
#pragma omp single
                {
                    double V = 0.0;
                    for (int64_t b = 0; b < nb; ++b) V += part[b];
                    volume[s + 1] = V;
                }
            }
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < 2 * ne; ++i)
            Uavg[i] = sum[i] / (double)nsub + theta / (double)nsub * (U[i] - U0[i]);
    }
    free(Un); free(U0); free(sum); free(phi); free(part); free(row); free(slot); free(cur);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Barotropic viscous regularization, eq. (eq:viscosity_BT):                 */
/*   R^hV = div(H A grad(U / H))                                             */
/* integrated over each triangle as a sum of two-point fluxes through its     */
/* edges shared with another triangle (no viscous flux through coastlines):   */
/*   V_e = (1/A_e) sum_j H_j A_j (u_n - u_e) l_j / d_j,   u = U / H_e         */
/* with H_e the triangle mean of H0 + eta (as in the transport update), H_j   */
/* the mean of H0 + eta at the edge's two vertices, l_j the edge length, d_j  */
/* the distance between the two centroids, and the coefficient a background   */
/* value plus a part proportional to the velocity difference across the      */
/* edge (Sec. 2.2, after eq. (eq:viscosity_BT)): A_j = A0 + Cv l_j |u_n - u_e|. */
/* Local edge j of triangle (t0, t1, t2) joins t_j and t_{(j+1) mod 3}.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t lo, hi;
    int64_t slot;   /* 3 e + j */
} orc_edge;

static int cmp_edge(const void *a, const void *b)
{
    const orc_edge *p = (const orc_edge *)a, *q = (const orc_edge *)b;
    if (p->lo != q->lo) return p->lo < q->lo ? -1 : 1;
    if (p->hi != q->hi) return p->hi < q->hi ? -1 : 1;
    return p->slot < q->slot ? -1 : (p->slot > q->slot ? 1 : 0);
}

/* nb[3 e + j] = the other triangle on local edge j of e, or -1 (coast). */
int orc_edge_neighbours(int64_t ne, const int32_t *tri, int32_t *nb)
{
    if (ne <= 0) return ORC_ERR_ARG;
    orc_edge *ed = (orc_edge *)malloc(sizeof(orc_edge) * 3 * ne);
    if (!ed) return ORC_ERR_OOM;
    for (int64_t e = 0; e < ne; ++e)
        for (int j = 0; j < 3; ++j) {
            int32_t a = tri[3 * e + j], b = tri[3 * e + (j + 1) % 3];
            ed[3 * e + j].lo = a < b ? a : b;
            ed[3 * e + j].hi = a < b ? b : a;
            ed[3 * e + j].slot = 3 * e + j;
        }
    qsort(ed, (size_t)(3 * ne), sizeof(orc_edge), cmp_edge);
    int status = ORC_OK;
    for (int64_t i = 0; i < 3 * ne;) {
        int64_t k = i + 1;
        while (k < 3 * ne && ed[k].lo == ed[i].lo && ed[k].hi == ed[i].hi) ++k;
        if (k - i == 1) {
            nb[ed[i].slot] = -1;
        } else if (k - i == 2) {
            nb[ed[i].slot] = (int32_t)(ed[i + 1].slot / 3);
            nb[ed[i + 1].slot] = (int32_t)(ed[i].slot / 3);
        } else {
            status = ORC_ERR_MESH;   /* an edge shared by more than two triangles */
            for (int64_t t = i; t < k; ++t) nb[ed[t].slot] = -1;
        }
        i = k;
    }
    free(ed);
    return status;
}

/* Vector from vertex p to vertex r in metres: planar differences wrapped across
 * periodic seams; on the sphere dlon wrapped and scaled by R cos(lat0), dlat by R. */
static void edge_vec(const double *x, const double *y, uint32_t flags, double px, double py,
                     double radius, double clat0, int32_t p, int32_t r, double *dx, double *dy)
{
    double ax = x[r] - x[p], ay = y[r] - y[p];
    if (flags & ORC_SPHERICAL) {
        ax = wrap_half(ax, 2.0 * 3.14159265358979323846);
        *dx = radius * clat0 * ax;
        *dy = radius * ay;
    } else {
        if (flags & ORC_PERIODIC_X) ax = wrap_half(ax, px);
        if (flags & ORC_PERIODIC_Y) ay = wrap_half(ay, py);
        *dx = ax;
        *dy = ay;
    }
}

/* Per local edge: l (length) and l/d (d: centroid distance), zero on coasts.
 * Both centroids are placed relative to the edge's first vertex p, in the metric
 * of the edge (on the sphere: cos of the mean latitude of its two vertices). */
int orc_visc_geometry(int64_t nv, int64_t ne, const double *x, const double *y,
                      const int32_t *tri, uint32_t flags, double period_x, double period_y,
                      double radius, const int32_t *nb, double *elen, double *lod)
{
    if (nv <= 0 || ne <= 0) return ORC_ERR_ARG;
    for (int64_t e = 0; e < ne; ++e)
        for (int j = 0; j < 3; ++j) {
            int64_t i = 3 * e + j;
            int32_t n = nb[i];
            elen[i] = 0.0;
            lod[i] = 0.0;
            if (n < 0) continue;
            int32_t p = tri[3 * e + j], q = tri[3 * e + (j + 1) % 3];
            double c0 = (flags & ORC_SPHERICAL) ? cos(0.5 * (y[p] + y[q])) : 1.0;
            double ex, ey;
            edge_vec(x, y, flags, period_x, period_y, radius, c0, p, q, &ex, &ey);
            double cex = 0.0, cey = 0.0, cnx = 0.0, cny = 0.0;
            for (int k = 0; k < 3; ++k) {
                double dx, dy;
                edge_vec(x, y, flags, period_x, period_y, radius, c0, p, tri[3 * e + k], &dx, &dy);
                cex += dx;
                cey += dy;
                edge_vec(x, y, flags, period_x, period_y, radius, c0, p, tri[3 * (int64_t)n + k],
                         &dx, &dy);
                cnx += dx;
                cny += dy;
            }
            double ddx = (cnx - cex) / 3.0, ddy = (cny - cey) / 3.0;
            double l = sqrt(ex * ex + ey * ey), d = sqrt(ddx * ddx + ddy * ddy);
            if (!(d > 0.0)) return ORC_ERR_MESH;
            elen[i] = l;
            lod[i] = l / d;
        }
    return ORC_OK;
}

static void visc_apply(const orc_mesh *m, const orc_visc *vs, int linear_h, const double *H0,
                       const double *eta, const double *U, double *V)
{
    for (int64_t e = 0; e < m->ne; ++e) {
        const int32_t *t = m->tri + 3 * e;
        double He = linear_h ? (H0[t[0]] + H0[t[1]] + H0[t[2]]) / 3.0
                             : ((H0[t[0]] + eta[t[0]]) + (H0[t[1]] + eta[t[1]]) +
                                (H0[t[2]] + eta[t[2]])) / 3.0;
        double ux = U[2 * e] / He, uy = U[2 * e + 1] / He;
        double sx = 0.0, sy = 0.0;
        for (int j = 0; j < 3; ++j) {
            int32_t n = vs->nb[3 * e + j];
            if (n < 0) continue;
            const int32_t *tn = m->tri + 3 * (int64_t)n;
            double Hn = linear_h ? (H0[tn[0]] + H0[tn[1]] + H0[tn[2]]) / 3.0
                                 : ((H0[tn[0]] + eta[tn[0]]) + (H0[tn[1]] + eta[tn[1]]) +
                                    (H0[tn[2]] + eta[tn[2]])) / 3.0;
            int32_t p = t[j], q = t[(j + 1) % 3];
            double Hj = linear_h ? 0.5 * (H0[p] + H0[q])
                                 : 0.5 * ((H0[p] + eta[p]) + (H0[q] + eta[q]));
            double dux = U[2 * n] / Hn - ux, duy = U[2 * n + 1] / Hn - uy;
            double A = vs->A0 + vs->Cv * vs->elen[3 * e + j] * sqrt(dux * dux + duy * duy);
            double c = Hj * A * vs->lod[3 * e + j];
            sx += c * dux;
            sy += c * duy;
        }
        V[2 * e] = sx / m->Ae[e];
        V[2 * e + 1] = sy / m->Ae[e];
    }
}

/* V [ne][2] = R^hV(eta, U) as defined above (nb, elen, lod from the two
 * functions above; Ae from orc_geometry). */
int orc_visc_apply(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                   const int32_t *nb, const double *elen, const double *lod, double A0,
                   double Cv, int linear_h, const double *H0, const double *eta, const double *U,
                   double *V)
{
    if (nv <= 0 || ne <= 0 || !(A0 >= 0.0) || !(Cv >= 0.0)) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, NULL, NULL};
    orc_visc vs = {nb, elen, lod, A0, Cv};
    visc_apply(&m, &vs, linear_h, H0, eta, U, V);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SESM: the AB3-AM4 substep with dissipative coefficients (Sec. 2.2,        */
/* eqs. (eq4_7), (eq4_8)).  Per substep m, in the order of eq. (eq4_8):      */
/*   U_ab = (3/2 + beta) U^m - (1/2 + 2 beta) U^{m-1} + beta U^{m-2}         */
/*   eta^{m+1} = eta^m - dt_s (div U_ab + W)                                 */
/*   eta_am = delta eta^{m+1} + (1 - delta - gamma - zeta) eta^m             */
/*            + gamma eta^{m-1} + zeta eta^{m-2}                             */
/*   U^{m+1} = U^m + dt_s (-f e_z x U_ab - g H_am grad eta_am + R)           */
/* with H_am the triangle mean of H0 + eta_am (the depth of eq. (eq4_5) at   */
/* the AM4 level; mean H0 with linear_h).  Readings where the paper is       */
/* silent: the histories start from the initial state (U^{-1} = U^{-2} =    */
/* U^0, likewise eta), and the averaged transport is the mean of U_ab over   */
/* m = 0..M-1, the transport whose divergence the elevation sums over the    */
/* subcycle (the counterpart of eq. (eq4_11)).                               */
/* ------------------------------------------------------------------------ */
int orc_subcycle_sesm(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                      const double *gN, const double *Av, double g, double beta,
                      double delta, double gamma, double zeta, int linear_h,
                      const double *H0, const double *f, const double *R, const double *W,
                      int32_t nsub, double tau, double *eta, double *U, double *Uavg,
                      double *volume)
{
    if (nsub <= 0 || nv <= 0 || ne <= 0) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, gN, Av};
    double dts = tau / (double)nsub;
    size_t nb2 = sizeof(double) * 2 * ne, nbv = sizeof(double) * nv;
    double *U1 = (double *)malloc(nb2), *U2 = (double *)malloc(nb2), *Uab = (double *)malloc(nb2);
    double *e1 = (double *)malloc(nbv), *e2 = (double *)malloc(nbv), *enew = (double *)malloc(nbv);
    double *eam = (double *)malloc(nbv), *div = (double *)malloc(nbv);
    double *sum = (double *)calloc((size_t)(2 * ne), sizeof(double));
    if (!U1 || !U2 || !Uab || !e1 || !e2 || !enew || !eam || !div || !sum) {
        free(U1); free(U2); free(Uab); free(e1); free(e2); free(enew); free(eam); free(div);
        free(sum);
        return ORC_ERR_OOM;
    }
    memcpy(U1, U, nb2);
    memcpy(U2, U, nb2);
    memcpy(e1, eta, nbv);
    memcpy(e2, eta, nbv);
    if (volume) volume[0] = volume_of(&m, eta);
    for (int32_t s = 0; s < nsub; ++s) {
        /* AB3 transport */
        for (int64_t i = 0; i < 2 * ne; ++i)
            Uab[i] = (1.5 + beta) * U[i] - (0.5 + 2.0 * beta) * U1[i] + beta * U2[i];
        /* elevation from the divergence of the AB3 transport */
        for (int64_t v = 0; v < nv; ++v) div[v] = 0.0;
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k) div[tri[3 * e + k]] += slot_flux(&m, e, k, Uab + 2 * e);
        for (int64_t v = 0; v < nv; ++v)
            enew[v] = eta[v] - dts * (div[v] / Av[v] + (W ? W[v] : 0.0));
        /* AM4 elevation */
        for (int64_t v = 0; v < nv; ++v)
            eam[v] = delta * enew[v] + (1.0 - delta - gamma - zeta) * eta[v] + gamma * e1[v] +
                     zeta * e2[v];
        /* transport: explicit Coriolis on U_ab, pressure of eta_am */
        for (int64_t e = 0; e < ne; ++e) {
            orc_elem q;
            elem_quantities(&m, e, eam, H0, f[e], dts, linear_h, &q);
            const double *ua = Uab + 2 * e;
            double Unx = U[2 * e] + dts * (f[e] * ua[1] - g * q.He * q.gx + R[2 * e]);
            double Uny = U[2 * e + 1] + dts * (-f[e] * ua[0] - g * q.He * q.gy + R[2 * e + 1]);
            U2[2 * e] = U1[2 * e];
            U2[2 * e + 1] = U1[2 * e + 1];
            U1[2 * e] = U[2 * e];
            U1[2 * e + 1] = U[2 * e + 1];
            U[2 * e] = Unx;
            U[2 * e + 1] = Uny;
        }
        for (int64_t v = 0; v < nv; ++v) {
            e2[v] = e1[v];
            e1[v] = eta[v];
            eta[v] = enew[v];
        }
        for (int64_t i = 0; i < 2 * ne; ++i) sum[i] += Uab[i];
        if (volume) volume[s + 1] = volume_of(&m, eta);
    }
    for (int64_t i = 0; i < 2 * ne; ++i) Uavg[i] = sum[i] / (double)nsub;
    free(U1); free(U2); free(Uab); free(e1); free(e2); free(enew); free(eam); free(div); free(sum);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Consumer of the averaged transport (Sec. 2.3, eq. (eq4_13); Sec. 2.4):     */
/* K layers, thicknesses h at vertices (layer 0 at the surface), layer        */
/* transports on triangles.                                                   */
/*  1. z* target: h^{n+1}_k = h^0_k (H / H0), H = H0 + eta^{n+1}, per vertex.  */
/*  2. h^{n+1/2} = (h^n + h^{n+1}) / 2; on a triangle, the mean of its three   */
/*     vertices.                                                              */
/*  3. trim: U_k = U*_k - h^{n+1/2}_k / sum_j h^{n+1/2}_j                      */
/*               * (sum_j U*_j - <<U>>)                                       */
/*  4. diasurface velocity from the thickness equation, bottom up:            */
/*     w_bottom of the deepest layer is 0, and for each layer                 */
/*       w_top = w_bottom - (h^{n+1}_k - h^n_k)/tau - div U_k - W [k = 0],    */
/*     w[v][k] the velocity through the top of layer k, w[v][K] = 0.          */
/*     w[v][0] vanishes to rounding when the column thickness H0 + eta^{n+1}  */
/*     is the one the averaged transport carried (eq. (eq4_11)).              */
/* Readings: thickness of a layer on a triangle = mean of its vertices; W     */
/* enters the top layer; the divergence is the median-dual one of the         */
/* barotropic path.                                                           */
/* ------------------------------------------------------------------------ */
int orc_trim_zstar(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                   const double *gN, const double *Av, int32_t K, const double *H0,
                   const double *eta_new, const double *Uavg, const double *Ustar,
                   const double *hn, const double *h0, const double *W, double tau,
                   double *U, double *hnew, double *w)
{
    if (K <= 0 || nv <= 0 || ne <= 0 || !(tau > 0.0)) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, gN, Av};
    /* 1. z* target */
    for (int64_t v = 0; v < nv; ++v)
        for (int32_t k = 0; k < K; ++k)
            hnew[v * K + k] = h0[v * K + k] * ((H0[v] + eta_new[v]) / H0[v]);
    /* 2-3. trim per triangle */
    double *hh = (double *)malloc(sizeof(double) * K);
    double *div = (double *)malloc(sizeof(double) * nv * K);
    if (!hh || !div) {
        free(hh); free(div);
        return ORC_ERR_OOM;
    }
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *t = tri + 3 * e;
        double hs = 0.0, sx = 0.0, sy = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            double a = 0.5 * (hn[t[0] * K + k] + hnew[t[0] * K + k]);
            double b = 0.5 * (hn[t[1] * K + k] + hnew[t[1] * K + k]);
            double c = 0.5 * (hn[t[2] * K + k] + hnew[t[2] * K + k]);
            hh[k] = (a + b + c) / 3.0;
            hs += hh[k];
            sx += Ustar[(e * K + k) * 2];
            sy += Ustar[(e * K + k) * 2 + 1];
        }
        double ex = sx - Uavg[2 * e], ey = sy - Uavg[2 * e + 1];
        for (int32_t k = 0; k < K; ++k) {
            U[(e * K + k) * 2] = Ustar[(e * K + k) * 2] - hh[k] / hs * ex;
            U[(e * K + k) * 2 + 1] = Ustar[(e * K + k) * 2 + 1] - hh[k] / hs * ey;
        }
    }
    /* 4. layer divergences (ascending triangle order per vertex) and w */
    for (int64_t i = 0; i < nv * K; ++i) div[i] = 0.0;
    for (int64_t e = 0; e < ne; ++e)
        for (int j = 0; j < 3; ++j)
            for (int32_t k = 0; k < K; ++k)
                div[tri[3 * e + j] * K + k] += slot_flux(&m, e, j, U + (e * K + k) * 2);
    for (int64_t v = 0; v < nv; ++v) {
        w[v * (K + 1) + K] = 0.0;
        for (int32_t k = K - 1; k >= 0; --k)
            w[v * (K + 1) + k] = w[v * (K + 1) + k + 1] -
                                 (hnew[v * K + k] - hn[v * K + k]) / tau -
                                 div[v * K + k] / Av[v] - (k == 0 && W ? W[v] : 0.0);
    }
    free(hh);
    free(div);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Vertically integrated baroclinic forcing, eq. (eq4_4) (Sec. 2.1, end):      */
/*   R_e = sum_{k < nlev_e} (RA + RP + RhV)_k + tau_s - Cd |u_b| u_b            */
/* The vertical-viscosity tendencies of a column telescope to the stress at    */
/* the surface minus the stress at the bottom; the bottom stress is the        */
/* quadratic drag on the velocity of the element's deepest layer (Sec. 2.1).   */
/* RA, RP, RhV, u: [ne][K][2], any of RA/RP/RhV/tau_s may be NULL (term absent);*/
/* nlev NULL means K layers everywhere.  Layers at or beyond nlev_e are never  */
/* read.                                                                        */
/* ------------------------------------------------------------------------ */
int orc_forcing(int64_t ne, int32_t K, const int32_t *nlev, const double *RA,
                const double *RP, const double *RhV, const double *tau_s, const double *u,
                double Cd, double *R)
{
    if (ne <= 0 || K <= 0 || !(Cd >= 0.0) || (Cd > 0.0 && !u)) return ORC_ERR_ARG;
    for (int64_t e = 0; e < ne; ++e) {
        int32_t n = nlev ? nlev[e] : K;
        if (n < 1 || n > K) return ORC_ERR_ARG;
    }
    for (int64_t e = 0; e < ne; ++e) {
        int32_t n = nlev ? nlev[e] : K;
        for (int c = 0; c < 2; ++c) {
            double s = 0.0;
            for (int32_t k = 0; k < n; ++k) {
                size_t i = ((size_t)e * K + k) * 2 + c;
                double layer = 0.0;
                if (RA) layer += RA[i];
                if (RP) layer += RP[i];
                if (RhV) layer += RhV[i];
                s += layer;
            }
            if (tau_s) s += tau_s[2 * e + c];
            if (Cd > 0.0) {
                const double *ub = u + ((size_t)e * K + (n - 1)) * 2;
                double speed = sqrt(ub[0] * ub[0] + ub[1] * ub[1]);
                s -= Cd * speed * ub[c];
            }
            R[2 * e + c] = s;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Tangent-linear model: derivative of the subcycle map along                */
/* (d_eta0, d_U0, d_R, d_H0); the state is advanced alongside.               */
/* ------------------------------------------------------------------------ */
int orc_tlm(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
            const double *gN, const double *Av, double g, double theta, int linear_h,
            const double *H0, const double *f, const double *R, const double *W,
            int32_t nsub, double tau, const double *eta0, const double *U0,
            const double *d_eta0, const double *d_U0, const double *d_R,
            const double *d_H0, double *d_eta, double *d_U, double *d_Uavg)
{
    if (nsub <= 0) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, gN, Av};
    double dts = tau / (double)nsub;
    size_t nb2 = sizeof(double) * 2 * ne;
    double *eta = (double *)malloc(sizeof(double) * nv);
    double *U = (double *)malloc(nb2), *Un = (double *)malloc(nb2), *F = (double *)malloc(nb2);
    double *dUn = (double *)malloc(nb2), *dF = (double *)malloc(nb2);
    double *dsum = (double *)calloc((size_t)(2 * ne), sizeof(double));
    double *div = (double *)malloc(sizeof(double) * nv), *ddiv = (double *)malloc(sizeof(double) * nv);
    if (!eta || !U || !Un || !F || !dUn || !dF || !dsum || !div || !ddiv) return ORC_ERR_OOM;
    memcpy(eta, eta0, sizeof(double) * nv);
    memcpy(U, U0, nb2);
    memcpy(d_eta, d_eta0, sizeof(double) * nv);
    memcpy(d_U, d_U0, nb2);
    for (int32_t s = 0; s < nsub; ++s) {
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t *t = tri + 3 * e;
            const double *gg = gN + 6 * e;
            orc_elem q, dq;
            elem_quantities(&m, e, eta, H0, f[e], dts, linear_h, &q);
            /* tangent of the triangle quantities */
            double db = d_eta[t[1]] - d_eta[t[0]], dc = d_eta[t[2]] - d_eta[t[0]];
            dq.gx = db * gg[2] + dc * gg[4];
            dq.gy = db * gg[3] + dc * gg[5];
            if (linear_h)
                dq.He = (d_H0[t[0]] + d_H0[t[1]] + d_H0[t[2]]) / 3.0;
            else
                dq.He = ((d_H0[t[0]] + d_eta[t[0]]) + (d_H0[t[1]] + d_eta[t[1]]) +
                         (d_H0[t[2]] + d_eta[t[2]])) / 3.0;
            transport_update(&q, g, dts, U + 2 * e, R + 2 * e, Un + 2 * e);
            double al = q.al, den = 1.0 + al * al;
            const double *dU = d_U + 2 * e;
            double drx = dU[0] + al * dU[1] + dts * (-g * (dq.He * q.gx + q.He * dq.gx) + d_R[2 * e]);
            double dry = dU[1] - al * dU[0] + dts * (-g * (dq.He * q.gy + q.He * dq.gy) + d_R[2 * e + 1]);
            dUn[2 * e] = (drx + al * dry) / den;
            dUn[2 * e + 1] = (dry - al * drx) / den;
            for (int k = 0; k < 2; ++k) {
                F[2 * e + k] = (1.0 + theta) * Un[2 * e + k] - theta * U[2 * e + k];
                dF[2 * e + k] = (1.0 + theta) * dUn[2 * e + k] - theta * d_U[2 * e + k];
            }
        }
        for (int64_t v = 0; v < nv; ++v) { div[v] = 0.0; ddiv[v] = 0.0; }
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k) {
                div[tri[3 * e + k]] += slot_flux(&m, e, k, F + 2 * e);
                ddiv[tri[3 * e + k]] += slot_flux(&m, e, k, dF + 2 * e);
            }
        for (int64_t v = 0; v < nv; ++v) {
            eta[v] = eta[v] - dts * (div[v] / Av[v] + (W ? W[v] : 0.0));
            d_eta[v] = d_eta[v] - dts * (ddiv[v] / Av[v]);
        }
        for (int64_t i = 0; i < 2 * ne; ++i) {
            U[i] = Un[i];
            d_U[i] = dUn[i];
            dsum[i] += dUn[i];
        }
    }
    for (int64_t i = 0; i < 2 * ne; ++i)
        d_Uavg[i] = dsum[i] / (double)nsub + theta / (double)nsub * (d_U[i] - d_U0[i]);
    free(eta); free(U); free(Un); free(F); free(dUn); free(dF); free(dsum); free(div); free(ddiv);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: gradients of  <lam_eta, eta^M> + <lam_U, U^M> + <lam_Uavg, Uavg>  */
/* with respect to eta^0, U^0, R and H0.  The whole forward trajectory is    */
/* stored (no checkpointing in the oracle).  NULL seeds count as zero.       */
/* ------------------------------------------------------------------------ */
int orc_adjoint(int64_t nv, int64_t ne, const int32_t *tri, const double *Ae,
                const double *gN, const double *Av, double g, double theta, int linear_h,
                const double *H0, const double *f, const double *R, const double *W,
                int32_t nsub, double tau, const double *eta0, const double *U0,
                const double *lam_eta, const double *lam_U, const double *lam_Uavg,
                double *g_eta0, double *g_U0, double *g_R, double *g_H0)
{
    if (nsub <= 0) return ORC_ERR_ARG;
    orc_mesh m = {nv, ne, tri, Ae, gN, Av};
    double dts = tau / (double)nsub;
    double rM = 1.0 / (double)nsub;
    size_t nb2 = sizeof(double) * 2 * ne;
    double *etas = (double *)malloc(sizeof(double) * nv * (size_t)(nsub + 1));
    double *Us = (double *)malloc(nb2 * (size_t)(nsub + 1));
    double *F = (double *)malloc(nb2), *div = (double *)malloc(sizeof(double) * nv);
    double *le = (double *)malloc(sizeof(double) * nv), *le_new = (double *)malloc(sizeof(double) * nv);
    double *lU = (double *)malloc(nb2), *lU_new = (double *)malloc(nb2);
    if (!etas || !Us || !F || !div || !le || !le_new || !lU || !lU_new) return ORC_ERR_OOM;

    /* forward, storing every state */
    memcpy(etas, eta0, sizeof(double) * nv);
    memcpy(Us, U0, nb2);
    for (int32_t s = 0; s < nsub; ++s) {
        const double *eta = etas + (size_t)s * nv;
        const double *U = Us + (size_t)s * 2 * ne;
        double *etan = etas + (size_t)(s + 1) * nv;
        double *Un = Us + (size_t)(s + 1) * 2 * ne;
        for (int64_t e = 0; e < ne; ++e) {
            orc_elem q;
            elem_quantities(&m, e, eta, H0, f[e], dts, linear_h, &q);
            transport_update(&q, g, dts, U + 2 * e, R + 2 * e, Un + 2 * e);
            F[2 * e] = (1.0 + theta) * Un[2 * e] - theta * U[2 * e];
            F[2 * e + 1] = (1.0 + theta) * Un[2 * e + 1] - theta * U[2 * e + 1];
        }
        for (int64_t v = 0; v < nv; ++v) div[v] = 0.0;
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k) div[tri[3 * e + k]] += slot_flux(&m, e, k, F + 2 * e);
        for (int64_t v = 0; v < nv; ++v)
            etan[v] = eta[v] - dts * (div[v] / Av[v] + (W ? W[v] : 0.0));
    }

    /* seeds at m = M; Uavg = (1/M) sum_{m=1..M} U^m + (theta/M)(U^M - U^0) */
    for (int64_t v = 0; v < nv; ++v) le[v] = lam_eta ? lam_eta[v] : 0.0;
    for (int64_t i = 0; i < 2 * ne; ++i)
        lU[i] = (lam_U ? lam_U[i] : 0.0) + (lam_Uavg ? theta * rM * lam_Uavg[i] : 0.0);
    for (int64_t i = 0; i < 2 * ne; ++i) g_R[i] = 0.0;
    for (int64_t v = 0; v < nv; ++v) g_H0[v] = 0.0;

    for (int32_t s = nsub - 1; s >= 0; --s) {
        const double *eta = etas + (size_t)s * nv;
        const double *U = Us + (size_t)s * 2 * ne;
        /* U^{s+1} enters the running sum */
        if (lam_Uavg)
            for (int64_t i = 0; i < 2 * ne; ++i) lU[i] += rM * lam_Uavg[i];
        /* eta^{s+1} = eta^s - dts (D F + W): identity part */
        for (int64_t v = 0; v < nv; ++v) le_new[v] = le[v];
        for (int64_t i = 0; i < 2 * ne; ++i) lU_new[i] = 0.0;
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t *t = tri + 3 * e;
            const double *gg = gN + 6 * e;
            orc_elem q;
            elem_quantities(&m, e, eta, H0, f[e], dts, linear_h, &q);
            /* lam_F = -dts sum_k (lam_eta_k / A_k) S_{e,k} */
            double lFx = 0.0, lFy = 0.0;
            for (int k = 0; k < 3; ++k) {
                double w = -dts * le[t[k]] / Av[t[k]];
                lFx += w * (-Ae[e] * gg[2 * k]);
                lFy += w * (-Ae[e] * gg[2 * k + 1]);
            }
            /* F = (1+theta) U' - theta U */
            double lUnx = lU[2 * e] + (1.0 + theta) * lFx;
            double lUny = lU[2 * e + 1] + (1.0 + theta) * lFy;
            double lUox = -theta * lFx, lUoy = -theta * lFy;
            /* U' = C r,  C = (I + al J)^-1;  C^T = (I + al J) / (1 + al^2) */
            double al = q.al, den = 1.0 + al * al;
            double lrx = (lUnx - al * lUny) / den;
            double lry = (lUny + al * lUnx) / den;
            /* r = (I - al J) U + dts(-g He grad + R); (I - al J)^T = I + al J */
            lUox += lrx - al * lry;
            lUoy += lry + al * lrx;
            g_R[2 * e] += dts * lrx;
            g_R[2 * e + 1] += dts * lry;
            double lgx = -dts * g * q.He * lrx, lgy = -dts * g * q.He * lry;
            double lHe = -dts * g * (q.gx * lrx + q.gy * lry);
            for (int k = 0; k < 3; ++k) {
                le_new[t[k]] += gg[2 * k] * lgx + gg[2 * k + 1] * lgy;
                if (!linear_h) le_new[t[k]] += lHe / 3.0;
                g_H0[t[k]] += lHe / 3.0;
            }
            lU_new[2 * e] = lUox;
            lU_new[2 * e + 1] = lUoy;
        }
        memcpy(le, le_new, sizeof(double) * nv);
        memcpy(lU, lU_new, nb2);
    }
    if (lam_Uavg)
        for (int64_t i = 0; i < 2 * ne; ++i) lU[i] -= theta * rM * lam_Uavg[i];
    memcpy(g_eta0, le, sizeof(double) * nv);
    memcpy(g_U0, lU, nb2);
    free(etas); free(Us); free(F); free(div); free(le); free(le_new); free(lU); free(lU_new);
    return ORC_OK;
}
