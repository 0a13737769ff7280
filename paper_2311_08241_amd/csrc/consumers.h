// Argument blocks of the consumer and forcing kernels (consumers.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sesub {

// Consumer of the averaged transport (FP64): trim of K layer transports, z*
// thicknesses, diasurface velocity.  One wavefront per triangle / vertex, lane =
// layer (K <= 64).
struct TrimArgs {
    int64_t nv, ne;
    int32_t K;
    double tau;
    const int32_t *tri, *row_ptr, *pcol;
    const double *geom;         // 5 SoA arrays [ne]: gbx gby gcx gcy A_e
    const double *Av;
    const double *H0, *eta_new, *Uavg, *Ustar, *hn, *h0, *W;
    double *U, *hnew, *w;
    // tile form only (the mesh's trim tiles): headers [ntiles][8], halo vertices, local
    // triangle records, local triangle of each CSR entry; local vertex capacity
    const int32_t *tt_hdr, *tt_lv;
    const int2 *tt_le;
    const uint16_t *tt_rloc;
    int32_t tt_ntiles, tt_cap_v;
};
// S: per-triangle sub-cell flux vectors [ne][3][2], S_k = -A_e grad N_k
hipError_t launch_trim(const TrimArgs &a, const double *S, hipStream_t s);
// Tile form: triangles (local ones) per tile and local vertices per tile for K layers
int trim_tile_cap_e(int K);
int trim_tile_cap_v(int K);
constexpr int kTrimTileOwn = 64;   // own vertices per tile
hipError_t launch_trim_tile(const TrimArgs &a, const double *S, hipStream_t s);

// Barotropic viscous term: V = div(H A grad(U / H)) per triangle (two-point fluxes
// through edges shared with a neighbour); out = base + sign V (base may be null).
struct ViscArgs {
    int64_t ne;
    const int32_t *tri;
    const int32_t *nb;          // [ne][4] neighbour across local edge j, -1 on coasts
    const void *vgeo;           // [ne][3][2] (l, l/d) in the path's precision
    const void *geom;           // 5 SoA arrays [ne] (A_e is the fifth)
    const void *H0, *eta, *U;   // eta: FP32 holds eta - eta_ref
    void *ubar;                 // [ne][2] scratch: U / H_e
    const void *base;           // [ne][2] or null
    void *out;                  // [ne][2]
    double A0, Cv, eta_ref;
    int32_t linear_h;
    int32_t sign;               // +1 or -1
};
hipError_t launch_visc(bool f32, const ViscArgs &a, hipStream_t s);

struct ForcingArgs {
    int64_t ne;
    int32_t K;
    int32_t out_f32;
    double Cd;
    const int32_t *nlev;        // [ne] or null (K everywhere)
    const double *RA, *RP, *RhV, *u;   // [ne][K][2], any may be null
    const double *tau_s;        // [ne][2] or null
    void *R;                    // [ne][2] double or float
    uint32_t *faults;
};
hipError_t launch_forcing(const ForcingArgs &a, hipStream_t s);

}  // namespace sesub
