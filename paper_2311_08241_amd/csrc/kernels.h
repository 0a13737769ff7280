// Kernel-side argument blocks shared by kernels.hip and the host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sesub {

// Constants of one member's subcycle (one baroclinic step).
struct StepC {
    double dts, g, theta, opt, thM, Mdbl, eta_ref;   // opt = 1 + theta, thM = theta / M
    float dts_f, g_f, theta_f, opt_f, eta_ref_f, pad_f;
    int32_t nsub, flags, ntiles, chunk0;   // chunk0: first launch index of this member
    int64_t vol_off;    // offset of this member's volume partials
    // AB3-AM4 coefficients (SESM): U_ab = ab0 U^m - ab1 U^{m-1} + ab2 U^{m-2};
    // eta_am = am0 eta^{m+1} + am1 eta^m + am2 eta^{m-1} + am3 eta^{m-2}
    double ab0, ab1, ab2, am0, am1, am2, am3;
    float ab0_f, ab1_f, ab2_f, am0_f, am1_f, am2_f, am3_f, pad2_f;
};

enum : int32_t { KF_LINEAR_H = 1, KF_TRACK_VOLUME = 4 };

// Fixed-width deposit rows of the tile kernel: a vertex with at most this many
// triangles keeps its sub-cell fluxes at kEllWidth * (local vertex) + rank, the
// unused entries zero (odd, so that the rows of consecutive vertices fall in
// distinct LDS banks).
constexpr int kEllWidth = 7;

// Triangle slots per thread that can hold owned triangles (the first ones of the
// local order), for EPT slots in all: only these carry running-sum registers.
__host__ __device__ constexpr int own_slots(int ept) { return ept <= 2 ? ept : ept - 1; }

struct TileHdrK {   // mirror of TileHdr (same layout)
    int32_t vbase, nv0, ebase, nown, lv_off, le_off, cs_off, rw_off, member, mtile, p0, p1;
};

struct TileArgs {
    const TileHdrK *hdr;
    const int32_t *nV, *nE, *lv_gid;
    const uint32_t *le_rec;     // per local triangle, 4 words: global id, packed local
                                // vertices and flux positions (3 words)
    const uint16_t *cs_row;
    const void *lgeo;           // per local triangle: gbx, gby, gcx, gcy (4 values)
    const void *lae;            // per local triangle: A_e
    const void *lv_av;          // per local vertex: 1 / A_v
    const StepC *mem;           // per-member constants (batches); nullptr: use c0
    StepC c0;
    void *eta_u, *eta_w;        // ping-pong pair: member chunk ch reads (ch even ? u : w)
    void *U_u, *U_w;
    const void *R, *f, *H0, *W, *Av;
    const double *Av64;
    void *sum;                  // double2 running sum per triangle (both precisions)
    void *U0c;                  // copy of U^0
    double *Uavg;
    double *vol_part;
    uint32_t *faults;
    const int32_t *tile_list;   // tiles of this launch (nullptr: all ntiles)
    int32_t K, chunk, ntiles, xcd;
    int32_t ksub;               // substeps per launch (K; K / 2 with the viscous term)
    int32_t cap_nv, cap_ne, cap_nvu, cap_cs;
    int32_t ell;                // deposits in fixed-width rows (kEllWidth per vertex)
    // viscous term only: per local triangle the local neighbours across its three
    // edges (16 bits each, 0xffff: none in the tile) and (l, l/d) of the three edges
    const uint32_t *vnb;
    const void *vgeo;
    double vA0, vCv;
    // AB3-AM4 only: two sets of (eta, eta^{-1}, eta^{-2}, eta_am) and of
    // (U, U^{-1}, U_ab), global numbering; chunk ch writes set ch & 1 and reads
    // set (ch - 1) & 1 (the caller's eta_u / U_u at the member's first chunk)
    void *sm_v[2][4];
    void *sm_e[2][3];
    // forward-backward only (adjoint recompute): when set, the elevation of the owned
    // vertices after member substep m (m = 1 .. nsub - 1) is also written to
    // traj + m * traj_stride (global numbering)
    void *traj;
    int64_t traj_stride;
    // access policy: non-zero selects the kernel that streams the tile's own tables and
    // the write-back past the caches (meshes whose launch traffic exceeds what the
    // caches keep between launches)
    int32_t nt;
};

// Reverse (adjoint) substeps of the forward-backward scheme on a tile plan: one launch
// runs cnt reverse substeps, the substeps of trajectory slots s_hi - 1 down to
// s_hi - cnt, on a tile and cnt rings of halo (the forward tile kernel's rings).
struct AdjTileArgs {
    const TileHdrK *hdr;
    const int32_t *nV, *nE, *lv_gid;
    const uint32_t *le_rec;
    const uint16_t *cs_row;
    const void *lgeo, *lae;     // per local triangle: gbx gby gcx gcy; A_e
    const void *Av, *H0, *f;    // global numbering, the precision's type
    // forward elevation of slot s: s == 0 ? eta_s0 : traj + s * traj_stride
    const void *eta_s0, *traj;
    int64_t traj_stride;
    const void *lam_eta_in, *lam_U_in;   // adjoint state before the launch
    void *lam_eta_out, *lam_U_out;       // after (owned entries)
    const double *lam_Uavg;              // seed of <<U>> or nullptr
    void *gR, *gH0;                      // accumulated gradients (owned entries updated)
    StepC c;
    double rM;                           // 1 / M
    // seed != 0 (the sweep's first launch): the state before it is the seed itself —
    // lam_eta_in / lam_U_in are the caller's seeds or null for zero, the transport's
    // plus thrM <<U>>-seed — and the gradients start from zero.  fin != 0 (the last
    // launch): the transport's final value minus thrM <<U>>-seed, written to lam_U_out
    // and g_U0, the elevation's also to g_eta0 (either may be null)
    double thrM;                         // theta / M
    void *g_eta0, *g_U0;
    int32_t seed, fin;
    int32_t K, cnt, s_hi, ntiles, xcd, ell;
    int32_t cap_nv, cap_ne, cap_nvu, cap_cs;
};

struct PlainArgs {
    int64_t nv, ne;
    const int32_t *tri, *row_ptr, *pcol;
    const void *geom;           // 5 SoA arrays [ne]
    const void *H0, *R, *f, *W, *Av;
    const double *Av64;
    void *eta, *U, *phi, *sum, *U0c;
    // non-null: the plain step reads the state (eta, U) from here and writes eta and U
    // (out of place; the source is not modified)
    const void *eta_src, *U_src;
    double *Uavg, *vol_part;
    uint32_t *faults;
    StepC c;
    int32_t m;                  // substep index 0..nsub-1
    int32_t nblk_v;             // blocks of the vertex launch (volume row width)
    int32_t fwd_only;           // 1: state update only (no running sum, average, volume)
    // AB3-AM4 (SESM) only: histories, AM4 elevation, AB3 transport
    void *eta1, *eta2, *etaA, *U1, *U2, *Uab;
};

// Reverse (adjoint) substep: triangle gather then vertex CSR sum.
struct AdjArgs {
    int64_t nv, ne;
    const int32_t *tri, *row_ptr, *pcol;
    const void *geom;           // 5 SoA arrays [ne]
    const void *H0, *Av;
    const void *f;
    const void *eta_m;          // forward state eta^m
    void *lam_eta;              // in: lambda_eta^{m+1}; out: lambda_eta^m
    void *lam_U;                // in: lambda_U^{m+1};   out: lambda_U^m
    const double *lam_Uavg;     // seed of <<U>> or nullptr
    void *gR, *gH0;             // accumulated gradients (R: [ne][2], H0: [nv])
    void *psi;                  // [ne][4] scratch: three slot terms and lambda_H / 3
    StepC c;
    double rM, thrM;            // 1/M and theta/M
};

// Host launchers (kernels.hip)
// mode: 0 forward-backward, 1 AB3-AM4, 2 forward-backward with the viscous term
hipError_t launch_tile(bool f32, int mode, int ept, int block, const TileArgs &a, int grid,
                       size_t lds, hipStream_t s);
hipError_t launch_plain_step(bool f32, const PlainArgs &a, hipStream_t s);
hipError_t launch_vol_reduce(const double *part, int64_t width, int32_t rows, double add,
                             double *out, hipStream_t s);
hipError_t launch_adj_step(bool f32, const AdjArgs &a, hipStream_t s);
// A reverse substep (rev) and a forward state-only substep (fwd, fwd_only set) of the
// same mesh in two launches instead of four; the two must touch disjoint arrays.
hipError_t launch_adj_pair(bool f32, const AdjArgs &rev, const PlainArgs &fwd, hipStream_t s);
// lam_eta = seed or 0; lam_U = seed + thrM * lam_Uavg; gR = gH0 = 0
hipError_t launch_adj_init(bool f32, const AdjArgs &a, const void *seed_eta, const void *seed_U,
                           hipStream_t s);
// lam_U -= thrM * lam_Uavg; g_eta0 = lam_eta, g_U0 = lam_U where not null
hipError_t launch_adj_final(bool f32, const AdjArgs &a, void *g_eta0, void *g_U0, hipStream_t s);
// Raise the dynamic-LDS limit of a tile kernel instantiation (call before any
// stream capture that launches it).
hipError_t prepare_tile(bool f32, int mode, int ept, int block);
// Reverse tile kernel: LDS bytes, its limit raised (before any capture), launch.
int adj_tile_lds_bytes(bool f32, int block, int cnt, int cap_nv, int cap_nvu, int cap_cs);
hipError_t prepare_adj_tile(bool f32, int ept, int block);
hipError_t launch_adj_tile(bool f32, int ept, int block, const AdjTileArgs &a, size_t lds,
                           hipStream_t s);
// The reverse launch a and an independent recompute launch f (mode 3, the same plan) in
// one launch of a.ntiles + f.ntiles workgroups; lds: the larger of the two kernels' LDS.
hipError_t launch_adj_tile_pair(bool f32, int ept, int block, const AdjTileArgs &a,
                                const TileArgs &f, size_t lds, hipStream_t s);
hipError_t launch_sesm_step(bool f32, const PlainArgs &a, hipStream_t s);
int tile_lds_bytes(bool f32, bool sm, int block, int K, int cap_nv, int cap_ne, int cap_nvu,
                   int cap_cs);
hipError_t launch_sesm_fin(bool f32, const PlainArgs &a, hipStream_t s);

}  // namespace sesub
