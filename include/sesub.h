/*
 * sesub.h — C ABI of the MI355X (gfx950) barotropic subcycle library.
 *
 * The library advances the barotropic (external) mode of a split-explicit
 * ocean model over one baroclinic step with the dissipative forward-backward
 * scheme of Banerjee et al., arXiv 2311.08241, Sec. 2.2, eq. (eq4_10):
 *
 *   U^{m+1} = U^m - dt_s [ (f/2) e_z x (U^{m+1} + U^m) + g H^m grad eta^m - R ]
 *   eta^{m+1} = eta^m - dt_s [ div((1+theta) U^{m+1} - theta U^m) + W ]
 *
 * for m = 0..M-1, dt_s = tau/M, H^m = H0 + eta^m, R frozen (Sec. 2.2,
 * eq. (eq4_5); the pressure term carries the sign of eq. (eq4_5)), and returns
 * the averaged transport of eq. (eq4_12)
 *
 *   <<U>> = (1/M) sum_{m=1..M} U^m + (theta/M) (U^M - U^0).
 *
 * Scalars (eta, H0, W) live at mesh vertices, transports (U, R) and f on
 * triangles.  The gradient is the P1 gradient per triangle; the divergence is
 * the median-dual finite-volume divergence with no flux through coastlines.
 *
 * Conventions (all entry points):
 *  - Every function returns se_status; SE_OK is 0.  Nothing aborts or exits.
 *    se_last_error() returns a thread-local description of the last failure.
 *  - "device" pointers are HIP device memory of the device the mesh was
 *    created on; "host" pointers are ordinary host memory.  The library never
 *    frees caller memory.  Meshes, batches and plans own their own device
 *    arrays (allocated at creation or at se_set_plan, freed at destroy).
 *  - Field arrays are in the mesh's internal (reordered) numbering; the
 *    permutations from se_mesh_perm map it to the caller's numbering.
 *  - Element type follows se_params.precision: SE_F64 -> double for eta, U,
 *    R, f, H0, W; SE_F32_MIXED -> float for those, with eta stored as the
 *    deviation eta - eta_ref.  Uavg and volume are always double.
 *  - stream is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously; only se_check_faults and se_mesh_* copies synchronise.
 *  - Results in SE_F64 are bit-for-bit deterministic for any plan: no float
 *    atomics, fixed per-vertex summation order (ascending triangle index).
 */
#ifndef SESUB_H
#define SESUB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SE_OK = 0,
    SE_ERR_ARG = 1,         /* invalid argument (NULL, size, dtype, plan)            */
    SE_ERR_MESH = 2,        /* invalid mesh (index range, orientation, duplicate)    */
    SE_ERR_HIP = 3,         /* a HIP runtime call failed                             */
    SE_ERR_OOM = 4,         /* device or host allocation failed                      */
    SE_ERR_CFL = 5,         /* dt_s beyond the stability bound (SE_CHECK_CFL)        */
    SE_ERR_DRY = 6,         /* reserved: reported through se_check_faults            */
    SE_ERR_NONFINITE = 7,   /* reserved: reported through se_check_faults            */
    SE_ERR_UNSUPPORTED = 8  /* valid request the library does not implement         */
} se_status;

typedef enum { SE_F64 = 0, SE_F32_MIXED = 1 } se_precision;

/* Time-stepping scheme of the substeps (se_params.scheme).
 * SE_SCHEME_SE: the dissipative forward-backward substep of eq. (eq4_10)
 *   (the default; all entry points).
 * SE_SCHEME_SESM: the AB3-AM4 substep of Sec. 2.2, eqs. (eq4_7)-(eq4_8):
 *     U_ab = (3/2 + beta) U^m - (1/2 + 2 beta) U^{m-1} + beta U^{m-2}
 *     eta^{m+1} = eta^m - dt_s (div U_ab + W)
 *     eta_am = delta eta^{m+1} + (1 - delta - gamma - zeta) eta^m
 *              + gamma eta^{m-1} + zeta eta^{m-2}
 *     U^{m+1} = U^m + dt_s (-f e_z x U_ab - g H_am grad eta_am + R)
 *   with H_am = H0 + eta_am; the histories start from the initial state
 *   (U^{-1} = U^{-2} = U^0, likewise eta) and <<U>> is the mean of U_ab over
 *   m = 0..M-1 (the transport whose divergence the elevation sums).  The
 *   coefficients come from se_params (eq. (eqdp_6) gives the paper's
 *   settings); theta is not used.  Supported by se_subcycle (the tile kernel
 *   hands (eta, eta^{m-1}, eta^{m-2}, eta_am) and (U, U^{m-1}, U_ab) from launch
 *   to launch with the last transport update pending; a final kernel applies
 *   it) and se_subcycle_plain; the adjoint and the batched form return
 *   SE_ERR_UNSUPPORTED. */
typedef enum { SE_SCHEME_SE = 0, SE_SCHEME_SESM = 1 } se_scheme;

/* mesh flags */
#define SE_PERIODIC_X 1u
#define SE_PERIODIC_Y 2u
#define SE_SPHERICAL 4u

/* parameter flags */
#define SE_LINEAR_H 1u      /* H = H0 in the pressure term (linear free surface)     */
#define SE_CHECK_CFL 2u     /* reject dt_s above the scheme's stability bound        */
#define SE_TRACK_VOLUME 4u  /* write sum_v A_v eta_v after every substep             */

/* fault bits (se_check_faults) */
#define SE_FAULT_DRY 1u       /* a triangle saw H = mean(H0 + eta) <= 0              */
#define SE_FAULT_NONFINITE 2u /* eta became NaN or Inf                               */
#define SE_FAULT_LAYERS 4u    /* se_forcing_assemble met a layer count outside 1..K            */

typedef struct se_mesh se_mesh;
typedef struct se_batch se_batch;

/* Mesh description (host arrays, read only during se_mesh_create).
 * x, y [nv]: planar metres, or (longitude, latitude) in radians with
 * SE_SPHERICAL (sphere of the given radius; the local metric of a triangle
 * uses the cosine of its mean latitude).  tri [ne][3]: counter-clockwise
 * vertex triples.  Periodic directions wrap coordinate differences into
 * (-period/2, period/2]; longitude always wraps with period 2 pi. */
typedef struct {
    int64_t nv, ne;
    const double *x, *y;
    const int32_t *tri;
    uint32_t flags;
    double period_x, period_y, radius;
} se_mesh_desc;

/* Validate, reorder and upload a mesh (Sec. 2.1: scalars on vertices,
 * transports on triangles).  Vertices are sorted along a Hilbert curve on a
 * 2^16 x 2^16 quantisation of the coordinate bounding box (ties by input
 * index); each triangle is rotated so its smallest vertex comes first and
 * triangles are sorted lexicographically.  Computes FP64 geometry (areas,
 * basis gradients, median-dual areas) and a Gershgorin bound mu_max of the
 * spectrum of -div grad.  device: HIP device ordinal.
 * Errors: SE_ERR_ARG (NULL, nv/ne <= 0, nv >= 2^31), SE_ERR_MESH (index out
 * of range, repeated vertex, non-positive area, duplicate triangle),
 * SE_ERR_OOM, SE_ERR_HIP. */
se_status se_mesh_create(const se_mesh_desc *desc, int device, se_mesh **out);
void se_mesh_destroy(se_mesh *mesh);

/* Sizes and the Gershgorin bound of -div grad (1/m^2). */
se_status se_mesh_info(const se_mesh *mesh, int64_t *nv, int64_t *ne, int64_t *nnz,
                       double *mu_max);
/* Host copies: vperm[new] = input vertex, eperm[new] = input triangle. */
se_status se_mesh_perm(const se_mesh *mesh, int32_t *vperm, int32_t *eperm);
/* Host copies of the reordered triangles [ne][3] and the vertex->triangle
 * CSR: row_ptr [nv+1], col [3 ne] = (triangle << 2) | local slot, triangles
 * ascending within a row. */
se_status se_mesh_csr(const se_mesh *mesh, int32_t *tri, int32_t *row_ptr, int32_t *col);
/* Host copies of the element neighbours of the barotropic viscous term (computed
 * on the host here; see se_barotropic_visc): nb [ne][3] the triangle across local
 * edge j = (tri[j], tri[(j+1) mod 3]) or -1 on a coast, edge length l [ne][3] and
 * l / d [ne][3] (d: distance between the two centroids; 0 on coasts).  Any output
 * may be NULL.  Errors: SE_ERR_ARG (NULL mesh), SE_ERR_MESH (an edge shared by more
 * than two triangles). */
se_status se_mesh_neighbours(const se_mesh *mesh, int32_t *nb, double *l, double *lod);
/* Host copies of the FP64 geometry: Av [nv] median-dual areas, Ae [ne]
 * triangle areas, gN [ne][3][2] P1 basis gradients. */
se_status se_mesh_geometry(const se_mesh *mesh, double *Av, double *Ae, double *gN);

/* Run parameters (Sec. 2.2). */
typedef struct {
    double g;          /* gravity (m/s^2)                                           */
    double theta;      /* dissipation parameter of eq. (eq4_10); 0.14 in the paper  */
    int32_t precision; /* se_precision                                              */
    uint32_t flags;    /* SE_LINEAR_H | SE_CHECK_CFL | SE_TRACK_VOLUME              */
    double eta_ref;    /* SE_F32_MIXED: eta arrays hold eta - eta_ref               */
    double h_max;      /* SE_CHECK_CFL: bound on H0 + eta over the run (m)          */
    int32_t scheme;    /* se_scheme (zero: SE_SCHEME_SE)                            */
    int32_t reserved;  /* must be 0                                                 */
    double beta, delta, gamma, zeta;   /* SE_SCHEME_SESM coefficients, eq. (eq4_7)  */
    /* Barotropic viscous regularization, eq. (eq:viscosity_BT) (Sec. 2.2): on when
     * either is > 0 (both finite, >= 0).  Coefficient A = visc_A0 + visc_Cv l |du|
     * (m^2/s) on an edge of length l with velocity difference du (see
     * se_barotropic_visc).  The term is evaluated at every substep from (eta^m, U^m)
     * and its value at the start of the subcycle is subtracted from R.  SE_SCHEME_SE
     * only: se_subcycle_plain, and se_subcycle, whose tile plan then runs k_fused / 2
     * substeps per launch (a neighbour across an edge lies one ring further out; the
     * plan needs k_fused >= 2); the adjoint, the batched form and SE_SCHEME_SESM return
     * SE_ERR_UNSUPPORTED when it is on. */
    double visc_A0, visc_Cv;
} se_params;

/* State, device arrays, updated in place. */
typedef struct {
    void *eta;       /* [nv]  in: eta^0, out: eta^M (F32: deviation from eta_ref)   */
    void *U;         /* [ne][2] in: U^0, out: U^M                                   */
    double *Uavg;    /* [ne][2] out: <<U>> of eq. (eq4_12); may be NULL             */
    double *volume;  /* out: sum_v A_v eta_v (absolute eta), [nsub+1] entries with  */
                     /* SE_TRACK_VOLUME (entry m after substep m), else [2]          */
                     /* (initial, final); may be NULL                                */
} se_state;

/* Frozen forcing and parameters of the subcycle, device arrays. */
typedef struct {
    const void *R;   /* [ne][2] barotropic forcing R of eq. (eq4_5) (m^2/s^2)       */
    const void *f;   /* [ne]    Coriolis parameter (1/s)                            */
    const void *H0;  /* [nv]    resting depth (m)                                   */
    const void *W;   /* [nv]    freshwater flux, positive out of the ocean (m/s);   */
                     /*         NULL means zero                                     */
} se_forcing;

/* Device workspace (bytes) se_subcycle / se_subcycle_adjoint need for nsub
 * substeps with the mesh's current plan; ckpt_every only matters for the
 * adjoint (0 for the forward). */
se_status se_workspace_bytes(const se_mesh *mesh, const se_params *params, int32_t nsub,
                             int32_t ckpt_every, size_t *bytes);

/* One baroclinic step: nsub substeps of dt_s = dt / nsub (eq. (eq4_10)),
 * then <<U>> (eq. (eq4_12)).  The next step continues from the returned
 * (eta^M, U^M) (Sec. 2.3: U^0 of a subcycle is the last available transport).
 * workspace: device buffer of se_workspace_bytes, 256-byte aligned.
 * Errors (synchronous): SE_ERR_ARG, SE_ERR_CFL (with SE_CHECK_CFL when
 * dt_s sqrt(g h_max mu_max) > 2/sqrt(1+2 theta)), SE_ERR_HIP. */
se_status se_subcycle(se_mesh *mesh, const se_params *params, se_state *state,
                      const se_forcing *forcing, int32_t nsub, double dt, void *workspace,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): se_subcycle with the same
 * kernels and results, its workspace taken from a static device array of
 * SE_NOALLOC_SCRATCH_BYTES instead of a caller buffer.  The library holds one such
 * array on every device it runs on, until the process ends.  Nothing is allocated:
 * the mesh must already have a tile plan (se_set_plan, or an earlier se_subcycle
 * call), and with the viscous term its tables must already exist (an earlier
 * se_subcycle call with the term builds them).  All calls on one device share that
 * device's array and find the last call's contents in it (the subcycle writes every
 * part of its workspace before reading it, so nothing needs clearing); calls that
 * overlap on one device (several streams or host threads) race and must be
 * serialised by the caller.
 * Errors: as se_subcycle, plus SE_ERR_ARG when se_workspace_bytes for this mesh,
 * precision and nsub exceeds SE_NOALLOC_SCRATCH_BYTES, or when the plan or the
 * viscous tables are missing. */
#define SE_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)   /* 256 MiB per device */
se_status se_subcycle_noalloc(se_mesh *mesh, const se_params *params, se_state *state,
                              const se_forcing *forcing, int32_t nsub, double dt,
                              void *stream);

/* Same step on the two-kernel path (one triangle launch and one vertex
 * launch per substep, no temporal blocking): the plain baseline. */
se_status se_subcycle_plain(se_mesh *mesh, const se_params *params, se_state *state,
                            const se_forcing *forcing, int32_t nsub, double dt,
                            void *workspace, void *stream);

/* Adjoint of se_subcycle.  For the scalar
 *   J = <lam_eta, eta^M> + <lam_U, U^M> + <lam_Uavg, <<U>>>
 * (plain sums over array entries) writes dJ/d eta^0, dJ/d U^0, dJ/dR, dJ/dH0.
 * Seeds may be NULL (zero); outputs may be NULL (not computed).  The forward
 * trajectory is recomputed from checkpoints stored every ckpt_every substeps
 * (1 <= ckpt_every <= nsub); each segment's recompute runs in the same launches
 * as the reverse substeps of the segment after it.  eta0/U0 are the forward inputs and are not
 * modified.  Element types follow params.precision; lam_Uavg is double. */
se_status se_subcycle_adjoint(se_mesh *mesh, const se_params *params, const void *eta0,
                              const void *U0, const se_forcing *forcing, int32_t nsub,
                              double dt, int32_t ckpt_every, const void *lam_eta,
                              const void *lam_U, const double *lam_Uavg, void *g_eta0,
                              void *g_U0, void *g_R, void *g_H0, void *workspace,
                              void *stream);

/* Ensemble of independent meshes advanced together in one launch sequence.
 * Member arrays are concatenated in member order (vertex arrays by member
 * nv, triangle arrays by member ne); each member has its own nsub and dt.
 * The batch keeps its own copy of the member meshes' device data. */
se_status se_batch_create(se_mesh *const *members, int32_t n, se_batch **out);
void se_batch_destroy(se_batch *batch);
se_status se_batch_info(const se_batch *batch, int64_t *nv_total, int64_t *ne_total,
                        int64_t *vert_offset /* [n+1] */, int64_t *elem_offset /* [n+1] */);
se_status se_batch_workspace_bytes(const se_batch *batch, const se_params *params,
                                   const int32_t *nsub, size_t *bytes);
/* state->volume: [sum_i (nsub_i + 1)] with SE_TRACK_VOLUME, else [2 n];
 * member i's entries start at sum_{j<i} of its predecessors' counts.
 * use_graph != 0: capture the launch sequence in a hipGraph on first use for
 * these pointers and replay it afterwards. */
se_status se_subcycle_batched(se_batch *batch, const se_params *params, se_state *state,
                              const se_forcing *forcing, const int32_t *nsub,
                              const double *dt, int use_graph, void *workspace,
                              void *stream);

/* Execution plan of the temporally blocked kernel: tile = vertices per
 * tile (64..8192), k_fused = substeps per launch (1..8), block = threads per
 * workgroup (256, 512 or 1024).  Applies to a mesh (kind 0) or a batch (kind 1).
 * Returns SE_ERR_ARG if the plan does not fit the kernel's register or LDS
 * budget for this mesh. */
se_status se_set_plan(void *mesh_or_batch, int32_t kind, int32_t tile, int32_t k_fused,
                      int32_t block);
se_status se_get_plan(const void *mesh_or_batch, int32_t kind, int32_t *tile,
                      int32_t *k_fused, int32_t *block);

/* Statistics of a candidate plan, computed on the host without changing the
 * current plan (works on host-only meshes): number of tiles; triangles and
 * vertices held per tile (max); halo overhead = local triangles / triangles
 * and local vertices / vertices summed over tiles; LDS bytes per workgroup
 * for FP32 and FP64; register tier (triangles per thread); modelled device
 * memory bytes per vertex-substep for FP32 and FP64 (compulsory traffic of
 * one launch of k_fused substeps divided by vertices x k_fused).  ok[0] / ok[1]
 * tell whether the plan runs in FP32 / FP64 without register spills.
 * Errors: SE_ERR_ARG when the plan is outside the limits of se_set_plan. */
typedef struct {
    int32_t ntiles, max_tri, max_vtx, tri_per_thread;
    int32_t lds_f32, lds_f64, ok_f32, ok_f64;
    double tri_overhead, vtx_overhead, bytes_per_vs_f32, bytes_per_vs_f64;
    /* the same budget for the AB3-AM4 scheme (three more vertex arrays in LDS,
     * two more transports per triangle in registers) */
    int32_t lds_sesm_f32, lds_sesm_f64, ok_sesm_f32, ok_sesm_f64;
} se_plan_stats_t;
se_status se_plan_stats(const void *mesh_or_batch, int32_t kind, int32_t tile, int32_t k_fused,
                        int32_t block, se_plan_stats_t *stats);

/* Synchronise the stream and return (and clear) the fault bits set by the
 * kernels since the last call: SE_FAULT_DRY, SE_FAULT_NONFINITE. */
se_status se_check_faults(void *mesh_or_batch, int32_t kind, void *stream,
                          uint32_t *fault_bits);

/* Consumer of the averaged transport (Sec. 2.3, eq. (eq4_13); Sec. 2.4,
 * z* coordinate), FP64, K layers (1 <= K <= 64; layer 0 at the surface):
 *   z* target      hnew[v][k] = h0[v][k] (H / H0[v]),  H = H0[v] + eta_new[v]
 *   mid thickness  h[k] on a triangle = mean over its vertices of (hn + hnew) / 2
 *   trim           U[e][k] = Ustar[e][k] - h[k] / sum_j h[j] (sum_j Ustar[e][j] - Uavg[e])
 *   diasurface velocity from the thickness equation, bottom up:
 *                  w[v][K] = 0,  w[v][k] = w[v][k+1] - (hnew - hn)[v][k] / tau
 *                                 - (div U[.][k])[v] - W[v] (k = 0 only)
 * with the median-dual divergence of the subcycle.  w[v][k] is the velocity
 * through the top of layer k; w[v][0] vanishes to rounding when eta_new and Uavg
 * come from the same subcycle (eq. (eq4_11)).  Device arrays, mesh numbering:
 * H0, eta_new [nv] (absolute eta), Uavg [ne][2], Ustar and U [ne][K][2] (U may
 * alias Ustar; no other output may alias an input), hn, h0, hnew [nv][K], W [nv] or
 * NULL, w [nv][K+1].  The first call on a mesh builds a table of its sub-cell flux
 * vectors on the host and uploads it synchronously (48 bytes per triangle, device
 * memory owned by the mesh).  With U distinct from Ustar the call is one launch over
 * tiles (runs of consecutive vertices with every triangle of their rows, at most 256,
 * 128, 96 or 64 triangles for K <= 8, <= 24, <= 32, <= 64); the first such call for
 * a class of K builds the mesh's tile tables, likewise synchronously (about 20 bytes
 * per triangle).  With U = Ustar, or when one vertex's row exceeds a tile, the call
 * runs as three launches, w serving as scratch between them; both forms give the
 * same bits.
 * Results equal the FP64 CPU definition to rounding: the sums over layers are
 * tree reductions and the vertical recursion a parallel suffix sum.
 * Errors: SE_ERR_ARG (NULL array, K outside 1..64, tau <= 0, host-only mesh). */
se_status se_trim_zstar(se_mesh *mesh, int32_t K, const double *H0, const double *eta_new,
                        const double *Uavg, const double *Ustar, const double *hn,
                        const double *h0, const double *W, double tau, double *U, double *hnew,
                        double *w, void *stream);

/* Barotropic viscous term of eq. (eq:viscosity_BT), R^hV = div(H A grad(U / H)),
 * per triangle e as a sum of two-point fluxes through its edges shared with
 * another triangle (no viscous flux through coasts):
 *   V[e] = (1/A_e) sum_j H_j A_j (l_j / d_j) (u_n - u_e),   u = U / H_e
 *   A_j  = A0 + Cv l_j |u_n - u_e|    (background plus a part proportional to the
 *                                      velocity difference across the edge)
 * H_e is the triangle mean of H0 + eta (mean H0 with SE_LINEAR_H), H_j the mean of
 * H0 + eta at the edge's two vertices, l_j the edge length and d_j the distance
 * between the centroids of e and its neighbour n.  precision SE_F64 or
 * SE_F32_MIXED (arrays of that type; eta of F32 holds eta - eta_ref); flags: only
 * SE_LINEAR_H is read.  Device arrays in mesh numbering: H0, eta [nv]; U, V [ne][2];
 * ws: scratch of 2 ne elements of the precision's type.  The first viscous call on
 * a mesh (and, for se_subcycle, the first after a plan change) builds and uploads
 * its neighbour tables synchronously; calls on one mesh must not run concurrently
 * from several host threads.
 * FP64 results follow the CPU definition operation for operation.
 * Errors: SE_ERR_ARG (NULL array, A0 or Cv negative or not finite, bad precision,
 * host-only mesh), SE_ERR_MESH (an edge shared by more than two triangles),
 * SE_ERR_OOM, SE_ERR_HIP. */
se_status se_barotropic_visc(se_mesh *mesh, int32_t precision, uint32_t flags, double eta_ref,
                             double A0, double Cv, const void *H0, const void *eta,
                             const void *U, void *V, void *ws, void *stream);

/* Vertically integrated baroclinic forcing of eq. (eq4_4) (Sec. 2.1, end), the
 * R the subcycle takes, per triangle e with nlev[e] layers (layer 0 at the surface):
 *   R[e] = sum_{k < nlev[e]} (RA + RP + RhV)[e][k] + tau_s[e] - Cd |u_b| u_b,
 *   u_b = u[e][nlev[e] - 1]
 * RA, RP, RhV: advective, pressure (without the eta part) and horizontal viscous
 * layer transport tendencies; the vertical viscous tendencies enter through their
 * column sum, surface stress minus bottom stress, with the quadratic drag on the
 * deepest layer's velocity as the bottom stress.  Device arrays, mesh triangle
 * numbering, FP64: RA, RP, RhV, u [ne][K][2]; tau_s [ne][2] (kinematic stress,
 * m^2/s^2); nlev [ne] int32.  Any of RA, RP, RhV, tau_s may be NULL (term absent);
 * nlev NULL means K layers everywhere; u may be NULL when Cd == 0.  Layers at or
 * below nlev[e] are never read.  R [ne][2] is written as double (SE_F64) or as the
 * float rounding of the FP64 sum (SE_F32_MIXED, the FP32 subcycle's R).
 * Results equal the FP64 CPU definition to rounding (the layer sum is a tree of
 * eight partial sums).  A triangle whose nlev lies outside 1..K gets NaN and sets
 * SE_FAULT_LAYERS (se_check_faults).
 * Errors: SE_ERR_ARG (R NULL, K < 1, Cd < 0 or not finite, Cd > 0 without u,
 * bad precision, host-only mesh), SE_ERR_HIP. */
se_status se_forcing_assemble(se_mesh *mesh, int32_t K, const int32_t *nlev, const double *RA,
                     const double *RP, const double *RhV, const double *tau_s, const double *u,
                     double Cd, int32_t precision, void *R, void *stream);

/* The AB3-AM4 (SE_SCHEME_SESM) coefficients of the paper's setting for the
 * dissipation of the forward-backward scheme with parameter theta (Sec. 2.2,
 * Sec. 3.2): chi = theta / 2 (eq. (eqdp_4), SE side: 2 chi = theta);
 * zeta = 0.010 - 0.135 chi and gamma = 0.083 - 0.514 chi (eq. (eqdp_6), second
 * line); delta = 2 chi + gamma + 2 zeta + 1/2 (eq. (eqdp_4), SESM side); beta as
 * given, or 0.281105 (the value with the largest stability range, Sec. 3.2) when
 * beta <= 0.  Host call, no device work.  out[4] receives beta, delta, gamma, zeta
 * (the order of se_params).  Errors: SE_ERR_ARG (out NULL, theta not finite). */
se_status se_sesm_coefficients(double theta, double beta, double *out);

/* Thread-local text of the last error. */
const char *se_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SESUB_H */
