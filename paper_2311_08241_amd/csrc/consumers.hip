// HIP kernels (gfx950, wave64) that consume the subcycle's results or prepare its
// forcing (Banerjee et al., arXiv 2311.08241):
//   trim of K layer transports to the averaged transport and z* thicknesses with
//     the diasurface velocity (Sec. 2.3, eq. (eq4_13); Sec. 2.4);
//   the barotropic viscous term of eq. (eq:viscosity_BT) (Sec. 2.2);
//   the vertically integrated baroclinic forcing of eq. (eq4_4) (Sec. 2.1).
// Compiled, like the subcycle kernels, without FMA contraction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "consumers.h"
#include "device_common.h"

namespace sesub {

namespace {

// ---------------------------------------------------------------------------
// Consumer of the averaged transport (FP64): z* target h0 (H / H0), mid thickness
// on triangles, trim of the layer transports to <<U>>, layer divergences in
// ascending triangle order, and the diasurface velocity from the bottom up.  One
// launch of k_trim_tile (below) when U is distinct from U* and every row fits a tile;
// otherwise three launches:
//   k_zstar_h       h^{n+1} = h0 (H0 + eta) / H0, one thread per vertex-layer; also
//                   hn + h^{n+1}, parked in w until k_zstar_w overwrites it
//   k_trim          8 lanes per triangle, 8 triangles per wavefront iteration;
//                   lane g holds layers g, g + 8, ...: 6 x the mid thickness (the
//                   common factor cancels in the trim weights), layer sums by
//                   butterflies over the 8 lanes, trimmed transports
//   k_zstar_w       8 lanes per vertex in the same layer layout: the CSR row's
//                   fluxes a few triangles at a time (all loads of a batch in
//                   flight), then w by suffix sums over the lanes, bottom up
// Every access of a group reads 8 consecutive layers (64 or 128 contiguous bytes).
// Results equal the definition to rounding (tree sums, reciprocals), not bit for bit.
// ---------------------------------------------------------------------------
// Also parks hn + hnew of every vertex-layer in w (same [v][k] place, row stride
// K + 1) for k_trim; k_zstar_w overwrites it with the diasurface velocity.
__global__ void __launch_bounds__(256) k_zstar_h(TrimArgs a) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.nv * a.K) return;
    const int64_t v = i / a.K;
    const double h = a.h0[i] * ((a.H0[v] + a.eta_new[v]) / a.H0[v]);
    a.hnew[i] = h;
    a.w[i + v] = a.hn[i] + h;
}

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each XCD owns
// one contiguous eighth of the ranges (neighbouring elements then share an L2).
__device__ __forceinline__ int64_t xcd_block() {
    const int G = gridDim.x, b = blockIdx.x, x = b & 7, q = b >> 3;
    const int base = G >> 3, rem = G & 7;
    return static_cast<int64_t>(x) * base + (x < rem ? x : rem) + q;
}

// Groups of 8 lanes (aligned in each row of 16) share one element; lane g of a group
// holds layers g, g + 8, g + 16, ...  Butterflies over the group by DPP: exchange with
// lane g ^ 1 and g ^ 2 (quad permutations), then with the mirrored lane 7 - g of the
// other quad (row_half_mirror), whose running total equals that of g ^ 4.
template <int CTRL> __device__ __forceinline__ double dpp64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // row_half_mirror: lane 7 - g of each 8

// Sum over the group, the same bits in all 8 lanes (each step adds two equal partial
// sums in either order).
__device__ __forceinline__ double grp_sum(double v) {
    v += dpp64<DPP_XOR1>(v);
    v += dpp64<DPP_XOR2>(v);
    return v + dpp64<DPP_HALF_MIRROR>(v);
}

// Inclusive suffix sum over the group (lane g: sum over g' >= g) and the group total.
__device__ __forceinline__ double grp_suffix(double v, int g, double &tot) {
    double s = v;
    double y = dpp64<DPP_XOR1>(v);
    if (!(g & 1)) s += y;
    v += y;
    y = dpp64<DPP_XOR2>(v);
    if (!(g & 2)) s += y;
    v += y;
    y = dpp64<DPP_HALF_MIRROR>(v);
    if (!(g & 4)) s += y;
    tot = v + y;
    return s;
}

// Blocks of 8 elements dealt to the wavefronts of each XCD in turn (workgroups go
// round-robin to the 8 XCDs; the grid is a multiple of 8 and small enough to be
// resident at once): the wavefronts of an XCD work on one compact window that moves
// along that XCD's eighth of the range, so elements sharing vertices (neighbours
// along the curve) meet in the XCD's L2 before streaming data evicts them.
struct Sweep {
    int64_t blk, step, lim;
};
__device__ __forceinline__ Sweep xcd_sweep(int64_t n) {
    const int G = gridDim.x, b = blockIdx.x, x = b & 7;
    const int wpb = blockDim.x >> 6;
    const int64_t gx = (G - x + 7) >> 3;   // workgroups on XCD x
    const int64_t wx = static_cast<int64_t>(b >> 3) * wpb +
                       __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t nblk = (n + 7) >> 3;
    return {nblk * x / 8 + wx, gx * wpb, nblk * (x + 1) / 8};
}

// Streaming accesses (each byte once): non-temporal, leaving L2 to the shared rows.
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ d2v ld_stream(const double *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
}
__device__ __forceinline__ void st_stream(double *p, d2v v) {
    __builtin_nontemporal_store(v, reinterpret_cast<d2v *>(p));
}

// L = ceil(K / 8) layers per lane.  Eight triangles per wavefront iteration: 6 x the
// mid thickness per layer (hn + hnew summed over the three vertices; the common factor
// cancels in the weights), the layer sums of thickness and transport by group sums,
// then the trimmed transport of each layer.
template <int L>
__global__ void __launch_bounds__(256) k_trim(TrimArgs a) {
    const int lane = threadIdx.x & 63, g = lane & 7, slot = lane >> 3;
    const int K = a.K;
    const int64_t ne = a.ne;
    const Sweep sw = xcd_sweep(ne);
    if (sw.blk >= sw.lim) return;
    // vertex indices of this lane's triangle, loaded one block ahead; past the end of
    // the range the last triangle stands in (its results are not stored)
    int64_t ec = min(8 * sw.blk + slot, ne - 1);
    int32_t ta = a.tri[3 * ec], tb = a.tri[3 * ec + 1], tc = a.tri[3 * ec + 2];
    for (int64_t bk = sw.blk; bk < sw.lim; bk += sw.step) {
        const bool live = 8 * bk + slot < ne;
        double hh[L], ux[L], uy[L];
        double hs = 0.0, sx = 0.0, sy = 0.0;
        const double *wa = a.w + static_cast<int64_t>(ta) * (K + 1);
        const double *wb = a.w + static_cast<int64_t>(tb) * (K + 1);
        const double *wc = a.w + static_cast<int64_t>(tc) * (K + 1);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = 8 * l + g;
            hh[l] = 0.0;
            ux[l] = 0.0;
            uy[l] = 0.0;
            if (k < K) {
                hh[l] = (wa[k] + wb[k]) + wc[k];
                const d2v u = ld_stream(a.Ustar + 2 * (ec * K + k));
                ux[l] = u.x;
                uy[l] = u.y;
            }
        }
        const int64_t bn = bk + sw.step;
        const int64_t en = bn < sw.lim ? min(8 * bn + slot, ne - 1) : ec;
        const int32_t na = a.tri[3 * en], nb = a.tri[3 * en + 1], nc = a.tri[3 * en + 2];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            hs += hh[l];
            sx += ux[l];
            sy += uy[l];
        }
        hs = grp_sum(hs);
        const double ex = grp_sum(sx) - a.Uavg[2 * ec];
        const double ey = grp_sum(sy) - a.Uavg[2 * ec + 1];
        const double rh = 1.0 / hs;
        if (live) {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const int k = 8 * l + g;
                if (k < K) {
                    const double q = hh[l] * rh;
                    d2v r;
                    r.x = ux[l] - q * ex;
                    r.y = uy[l] - q * ey;
                    st_stream(a.U + 2 * (ec * K + k), r);
                }
            }
        }
        ec = en;
        ta = na;
        tb = nb;
        tc = nc;
    }
}

// Eight vertices per wavefront iteration, CSR entries DB at a time (all their loads in
// flight): per layer the flux of the trimmed transport through the vertex's sub-cell
// boundary, then t_k = (hnew - hn) / tau + div_k / A_v (+ W at the top) and
// w_k = -(t_k + ... + t_{K-1}) by group suffix sums, layer blocks from the bottom up.
// The next block's row bounds and first 8 CSR columns (one per lane of the group,
// passed to the others by lane shuffles) are loaded while this block gathers.  Plain
// (temporal) accesses here: the 328-byte rows of w are not line aligned.
constexpr int ZW_DB = 3;

template <int L>
__global__ void __launch_bounds__(256) k_zstar_w(TrimArgs a, const double *S) {
    const int lane = threadIdx.x & 63, g = lane & 7, slot = lane >> 3;
    const int gbase = lane & ~7;
    const int K = a.K;
    const double inv_tau = 1.0 / a.tau;
    const double2 *U2 = reinterpret_cast<const double2 *>(a.U);
    const double2 *S2 = reinterpret_cast<const double2 *>(S);
    const int64_t nv = a.nv;
    const Sweep sw = xcd_sweep(nv);
    if (sw.blk >= sw.lim) return;
    // row bounds of this lane's vertex and entry g of its CSR row (the group's lanes
    // hold the first 8 entries), loaded a block ahead
    int64_t vc = min(8 * sw.blk + slot, nv - 1);
    int32_t j0 = a.row_ptr[vc], j1 = a.row_ptr[vc + 1];   // j1 > j0: no empty rows
    int32_t pq = a.pcol[min(j0 + g, j1 - 1)];
    for (int64_t bk = sw.blk; bk < sw.lim; bk += sw.step) {
        const bool live = 8 * bk + slot < nv;
        double dh[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = 8 * l + g;
            dh[l] = k < K ? (a.hnew[vc * K + k] - a.hn[vc * K + k]) * inv_tau : 0.0;
        }
        const int64_t bn = bk + sw.step;
        const int64_t vn = bn < sw.lim ? min(8 * bn + slot, nv - 1) : vc;
        const int32_t n0 = a.row_ptr[vn], n1 = a.row_ptr[vn + 1];
        double div[L];
#pragma unroll
        for (int l = 0; l < L; ++l) div[l] = 0.0;
        const int len = j1 - j0;
        for (int q0 = 0; q0 < len; q0 += ZW_DB) {
            double2 sv[ZW_DB];
            double2 F[ZW_DB][L];
#pragma unroll
            for (int q = 0; q < ZW_DB; ++q) {
                const int qq = min(q0 + q, len - 1);
                const int32_t pc = qq < 8 ? __shfl(pq, gbase + min(qq, 7), 64) : a.pcol[j0 + qq];
                sv[q] = S2[pc];
                const int64_t eK = static_cast<int64_t>(pc / 3) * K;
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    const int k = 8 * l + g;
                    F[q][l] = k < K ? U2[eK + k] : make_double2(0.0, 0.0);
                }
            }
#pragma unroll
            for (int q = 0; q < ZW_DB; ++q)
                if (q0 + q < len)
#pragma unroll
                    for (int l = 0; l < L; ++l)
                        div[l] += F[q][l].x * sv[q].x + F[q][l].y * sv[q].y;
        }
        const int32_t pn = a.pcol[min(n0 + g, n1 - 1)];
        const double rA = 1.0 / a.Av[vc];
        const double Wv = a.W ? a.W[vc] : 0.0;
        double *w = a.w + vc * (K + 1);
        double run = 0.0;   // sum of t over the layer blocks below
#pragma unroll
        for (int l = L - 1; l >= 0; --l) {
            const int k = 8 * l + g;
            const double t = k < K ? dh[l] + div[l] * rA + (k == 0 ? Wv : 0.0) : 0.0;
            double tot;
            const double sfx = grp_suffix(t, g, tot);
            if (live && k < K) w[k] = -(sfx + run);
            run += tot;
        }
        if (live && g == 0) w[K] = 0.0;
        vc = vn;
        j0 = n0;
        j1 = n1;
        pq = pn;
    }
}

// ---------------------------------------------------------------------------
// Tile form of the consumer, one launch.  A workgroup (32 groups of 8 lanes, lane g of
// a group holding layers g, g + 8, ...) takes one run of consecutive vertices with
// every triangle of their CSR rows (TrimTiles):
//   1. hn + hnew of the tile's vertices to LDS; its own vertices also write hnew and
//      keep (hnew - hn) / tau; the rows' local triangle and flux vector per entry
//   2. the trim of each local triangle (TPG per group) into registers, stored to U
//      when the tile owns the triangle (a triangle of an earlier run's vertex is trimmed
//      there too, from the same inputs, to the same bits)
//   3. per block of 8 layers: the trimmed transports to LDS, then each own vertex's
//      layer divergences over its row in CSR order
//   4. w by group suffix sums, bottom up
// The arithmetic of k_zstar_h + k_trim + k_zstar_w in the same order (the same bits),
// without the parked sums and the second pass over U.  U* is read with ordinary loads
// (the tiles after it find the shared triangles in L2); U, hnew and w are written once.
// ---------------------------------------------------------------------------
constexpr int TT_VPG = kTrimTileOwn / 32;   // own vertices per group

// triangles per group: the trimmed transports of a group's triangles sit in registers
// (4 TPG L VGPRs); kept near 128 VGPRs so that four workgroups share a CU (at K = 40,
// 64-triangle tiles ran 8% faster than 96-triangle ones despite their larger halo)
template <int L> constexpr int trim_tpg() { return L <= 1 ? 8 : L <= 3 ? 4 : L <= 4 ? 3 : 2; }

template <int L, int TPG>
__global__ void __launch_bounds__(256) k_trim_tile(TrimArgs a, const double *S) {
    extern __shared__ __align__(16) double tsm[];
    const int tid = threadIdx.x, g = tid & 7, grp = tid >> 3;
    const int K = a.K;
    const int32_t *hd = a.tt_hdr + 8 * xcd_block();
    const int32_t v0 = hd[0], nvo = hd[1], nvl = hd[2], nel = hd[3], neo = hd[4];
    const int32_t lv_off = hd[5], le_off = hd[6], nent = hd[7];
    constexpr int CE = 32 * TPG;
    double *sP = tsm;                                                     // [cap_v][K]
    d2v *sU = reinterpret_cast<d2v *>(tsm + static_cast<size_t>(a.tt_cap_v) * K);   // [CE][8]
    d2v *sS = sU + CE * 8;                                               // [3 CE]
    uint16_t *sL = reinterpret_cast<uint16_t *>(sS + 3 * CE);             // [3 CE]
    const double inv_tau = 1.0 / a.tau;
    // the loads of steps 2 and 3 that do not wait for LDS, issued first: the local
    // triangles' records, transports U* and <<U>> (past the tile's last triangle a group
    // repeats it and stores nothing), the own vertices' row bounds
    d2v Ut[TPG][L];
    int64_t ge[TPG];
    int pk[TPG];
    double uax[TPG], uay[TPG];
#pragma unroll
    for (int q = 0; q < TPG; ++q) {
        const int2 rec = a.tt_le[le_off + min(grp + 32 * q, nel - 1)];
        ge[q] = rec.x;
        pk[q] = rec.y;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = 8 * l + g;
            Ut[q][l] = k < K ? *reinterpret_cast<const d2v *>(a.Ustar + 2 * (ge[q] * K + k))
                             : d2v{0.0, 0.0};
        }
        uax[q] = a.Uavg[2 * ge[q]];
        uay[q] = a.Uavg[2 * ge[q] + 1];
    }
    const int32_t jb = a.row_ptr[v0];
    int j0[TT_VPG], j1[TT_VPG];
#pragma unroll
    for (int q = 0; q < TT_VPG; ++q) {
        const int lv = grp + 32 * q;
        const int64_t v = v0 + min(lv, nvo - 1);
        j0[q] = a.row_ptr[v];
        j1[q] = lv < nvo ? a.row_ptr[v + 1] : j0[q];
    }
    // 1. vertex columns
    double dh[TT_VPG][L];
#pragma unroll
    for (int q = 0; q < TT_VPG; ++q) {
        const int lv = grp + 32 * q;
#pragma unroll
        for (int l = 0; l < L; ++l) dh[q][l] = 0.0;
        if (lv < nvo) {
            const int64_t v = v0 + lv;
            const double sc = (a.H0[v] + a.eta_new[v]) / a.H0[v];
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const int k = 8 * l + g;
                if (k < K) {
                    const double hn = a.hn[v * K + k];
                    const double h = a.h0[v * K + k] * sc;
                    a.hnew[v * K + k] = h;
                    sP[lv * K + k] = hn + h;
                    dh[q][l] = (h - hn) * inv_tau;
                }
            }
        }
    }
    for (int lv = nvo + grp; lv < nvl; lv += 32) {
        const int64_t v = a.tt_lv[lv_off + lv - nvo];
        const double sc = (a.H0[v] + a.eta_new[v]) / a.H0[v];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = 8 * l + g;
            if (k < K) {
                const double h = a.h0[v * K + k] * sc;
                sP[lv * K + k] = a.hn[v * K + k] + h;
            }
        }
    }
    const d2v *S2 = reinterpret_cast<const d2v *>(S);
    for (int i = tid; i < nent; i += 256) {
        sL[i] = a.tt_rloc[jb + i];
        sS[i] = S2[a.pcol[jb + i]];
    }
    __syncthreads();
    // 2. trim
#pragma unroll
    for (int q = 0; q < TPG; ++q) {
        const int la = pk[q] & 1023, lb = (pk[q] >> 10) & 1023, lc = pk[q] >> 20;
        double hh[L];
        double hs = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = 8 * l + g;
            hh[l] = k < K ? (sP[la * K + k] + sP[lb * K + k]) + sP[lc * K + k] : 0.0;
            hs += hh[l];
            sx += Ut[q][l].x;
            sy += Ut[q][l].y;
        }
        hs = grp_sum(hs);
        const double ex = grp_sum(sx) - uax[q];
        const double ey = grp_sum(sy) - uay[q];
        const double rh = 1.0 / hs;
        const bool own = grp + 32 * q < neo;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = 8 * l + g;
            const double qh = hh[l] * rh;
            d2v r;
            r.x = Ut[q][l].x - qh * ex;
            r.y = Ut[q][l].y - qh * ey;
            Ut[q][l] = r;
            if (own && k < K) st_stream(a.U + 2 * (ge[q] * K + k), r);
        }
    }
    // 3. layer divergences of the own vertices, one block of 8 layers at a time
    double div[TT_VPG][L];
#pragma unroll
    for (int q = 0; q < TT_VPG; ++q)
#pragma unroll
        for (int l = 0; l < L; ++l) div[q][l] = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
#pragma unroll
        for (int q = 0; q < TPG; ++q)
            if (grp + 32 * q < nel) sU[(grp + 32 * q) * 8 + g] = Ut[q][l];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TT_VPG; ++q)
            for (int jj = j0[q] - jb; jj < j1[q] - jb; ++jj) {
                const d2v sv = sS[jj];
                const d2v F = sU[sL[jj] * 8 + g];
                div[q][l] += F.x * sv.x + F.y * sv.y;
            }
        __syncthreads();
    }
    // 4. w from the bottom up
#pragma unroll
    for (int q = 0; q < TT_VPG; ++q) {
        const int lv = grp + 32 * q;
        if (lv >= nvo) continue;
        const int64_t v = v0 + lv;
        const double rA = 1.0 / a.Av[v];
        const double Wv = a.W ? a.W[v] : 0.0;
        double *w = a.w + v * (K + 1);
        double run = 0.0;
#pragma unroll
        for (int l = L - 1; l >= 0; --l) {
            const int k = 8 * l + g;
            const double t = k < K ? dh[q][l] + div[q][l] * rA + (k == 0 ? Wv : 0.0) : 0.0;
            double tot;
            const double sfx = grp_suffix(t, g, tot);
            if (k < K) w[k] = -(sfx + run);
            run += tot;
        }
        if (g == 0) w[K] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Barotropic viscous regularization: one thread per triangle.  k_visc_u stores the
// velocity U / H_e of every triangle; k_visc sums the two-point fluxes
// H_j A_j (l/d)_j (u_n - u_e) over the triangle's edges shared with a neighbour,
// A_j = A0 + Cv l_j |u_n - u_e|, H_j the mean depth at the edge's two vertices.
// Each edge flux is evaluated by both of its triangles with the same operations
// and opposite sign.  FP64 follows the CPU definition operation for operation.
// ---------------------------------------------------------------------------
template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_visc_u(ViscArgs a) {
    using T2 = typename Vec2<T>::type;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.ne) return;
    const T *H0 = static_cast<const T *>(a.H0);
    const T *eta = static_cast<const T *>(a.eta);
    const int32_t *t = a.tri + 3 * e;
    const T He = visc_tri_depth<T, F32>(a.linear_h, static_cast<float>(a.eta_ref), H0[t[0]],
                                        H0[t[1]], H0[t[2]], eta[t[0]], eta[t[1]], eta[t[2]]);
    const T2 u = static_cast<const T2 *>(a.U)[e];
    T2 r;
    r.x = u.x / He;
    r.y = u.y / He;
    static_cast<T2 *>(a.ubar)[e] = r;
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_visc(ViscArgs a) {
    using T2 = typename Vec2<T>::type;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.ne) return;
    const T *H0 = static_cast<const T *>(a.H0);
    const T *eta = static_cast<const T *>(a.eta);
    const T2 *ub = static_cast<const T2 *>(a.ubar);
    const T *vg = static_cast<const T *>(a.vgeo) + 6 * e;
    const int4 nb = *reinterpret_cast<const int4 *>(a.nb + 4 * e);
    const int32_t t[3] = {a.tri[3 * e], a.tri[3 * e + 1], a.tri[3 * e + 2]};
    const T2 ue = ub[e];
    const T A0 = static_cast<T>(a.A0), Cv = static_cast<T>(a.Cv);
    const float eref = static_cast<float>(a.eta_ref);
    T Hv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Hv[k] = visc_vtx_depth<T, F32>(a.linear_h, eref, H0[t[k]], eta[t[k]]);
    const int32_t nbs[3] = {nb.x, nb.y, nb.z};
    T sx = 0, sy = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int32_t n = nbs[j];
        if (n < 0) continue;
        const T2 un = ub[n];
        visc_edge<T>(A0, Cv, static_cast<T>(0.5) * (Hv[j] + Hv[(j + 1) % 3]), vg[2 * j],
                     vg[2 * j + 1], un.x - ue.x, un.y - ue.y, sx, sy);
    }
    const T Ae = static_cast<const T *>(a.geom)[4 * a.ne + e];
    T vx = sx / Ae, vy = sy / Ae;
    if (a.base) {
        const T2 b = static_cast<const T2 *>(a.base)[e];
        if (a.sign > 0) {
            vx = b.x + vx;
            vy = b.y + vy;
        } else {
            vx = b.x - vx;
            vy = b.y - vy;
        }
    }
    T2 r;
    r.x = vx;
    r.y = vy;
    static_cast<T2 *>(a.out)[e] = r;
}

// ---------------------------------------------------------------------------
// Vertically integrated baroclinic forcing: eight lanes per triangle column.  Lane
// j of a group adds the layers k = j, j + 8, ... (each group load is one 128-byte
// run of (x, y) pairs), the group then combines its eight partial sums by a
// butterfly, and its first lane adds the surface stress and the bottom drag.
// ---------------------------------------------------------------------------
constexpr int FG = 8;   // lanes per column

template <bool OUT32>
__global__ void __launch_bounds__(256) k_forcing(ForcingArgs a) {
    const int j = threadIdx.x & (FG - 1);
    const int64_t e = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / FG;
    if (e >= a.ne) return;   // whole groups leave together (256 is a multiple of FG)
    const int K = a.K;
    const int n = a.nlev ? a.nlev[e] : K;
    double rx, ry;
    if (n < 1 || n > K) {
        if (j == 0) set_fault(a.faults, 4u);
        rx = ry = __builtin_nan("");
    } else {
        double sx = 0.0, sy = 0.0;
        const int64_t base = e * K;
#pragma unroll 4
        for (int k = j; k < n; k += FG) {
            const int64_t i = (base + k) * 2;
            double lx = 0.0, ly = 0.0;
            if (a.RA) { const double2 v = *reinterpret_cast<const double2 *>(a.RA + i); lx += v.x; ly += v.y; }
            if (a.RP) { const double2 v = *reinterpret_cast<const double2 *>(a.RP + i); lx += v.x; ly += v.y; }
            if (a.RhV) { const double2 v = *reinterpret_cast<const double2 *>(a.RhV + i); lx += v.x; ly += v.y; }
            sx += lx;
            sy += ly;
        }
#pragma unroll
        for (int o = 1; o < FG; o <<= 1) {
            sx += __shfl_xor(sx, o, 64);
            sy += __shfl_xor(sy, o, 64);
        }
        if (a.tau_s) {
            sx += a.tau_s[2 * e];
            sy += a.tau_s[2 * e + 1];
        }
        if (a.Cd > 0.0) {
            const double2 ub = *reinterpret_cast<const double2 *>(a.u + (base + n - 1) * 2);
            const double sp = sqrt(ub.x * ub.x + ub.y * ub.y);
            sx -= a.Cd * sp * ub.x;
            sy -= a.Cd * sp * ub.y;
        }
        rx = sx;
        ry = sy;
    }
    if (j == 0) {
        if (OUT32) {
            float2 r;
            r.x = static_cast<float>(rx);
            r.y = static_cast<float>(ry);
            static_cast<float2 *>(a.R)[e] = r;
        } else {
            double2 r;
            r.x = rx;
            r.y = ry;
            static_cast<double2 *>(a.R)[e] = r;
        }
    }
}

}  // namespace

hipError_t launch_visc(bool f32, const ViscArgs &a, hipStream_t s) {
    if (a.ne <= 0) return hipSuccess;
    const unsigned g = static_cast<unsigned>((a.ne + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL((k_visc_u<float, true>), dim3(g), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_visc<float, true>), dim3(g), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_visc_u<double, false>), dim3(g), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_visc<double, false>), dim3(g), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_forcing(const ForcingArgs &a, hipStream_t s) {
    if (a.ne <= 0) return hipSuccess;
    const unsigned g = static_cast<unsigned>((a.ne * FG + 255) / 256);
    if (a.out_f32) hipLaunchKernelGGL(k_forcing<true>, dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_forcing<false>, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Grids of 4 (k_trim) and 3 (k_zstar_w) workgroups per CU, all resident at once: the
// fastest of 2 to 7 per CU on a 2.2M-vertex, 40-layer mesh (fewer wavefronts per XCD
// keep the sweep's window, and its rows, inside L2; more overlap more loads).
template <int L> void launch_trim_layers(const TrimArgs &a, const double *S, hipStream_t s) {
    if (a.ne > 0) hipLaunchKernelGGL(k_trim<L>, dim3(256 * 4), dim3(256), 0, s, a);
    if (a.nv > 0) hipLaunchKernelGGL(k_zstar_w<L>, dim3(256 * 3), dim3(256), 0, s, a, S);
}

int trim_tile_cap_e(int K) {
    switch ((K + 7) / 8) {
        case 1: return 32 * trim_tpg<1>();
        case 2: return 32 * trim_tpg<2>();
        case 3: return 32 * trim_tpg<3>();
        case 4: return 32 * trim_tpg<4>();
        case 5: return 32 * trim_tpg<5>();
        case 6: return 32 * trim_tpg<6>();
        case 7: return 32 * trim_tpg<7>();
        default: return 32 * trim_tpg<8>();
    }
}
int trim_tile_cap_v(int K) { return trim_tile_cap_e(K); }

template <int L> hipError_t launch_trim_tile_l(const TrimArgs &a, const double *S, hipStream_t s) {
    constexpr int TPG = trim_tpg<L>();
    constexpr int CE = 32 * TPG;
    const size_t lds = static_cast<size_t>(a.tt_cap_v) * a.K * 8 + CE * (8 * 16 + 3 * 16 + 3 * 2);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(k_trim_tile<L, TPG>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds));
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_trim_tile<L, TPG>), dim3(a.tt_ntiles), dim3(256), lds, s, a, S);
    return hipGetLastError();
}

hipError_t launch_trim_tile(const TrimArgs &a, const double *S, hipStream_t s) {
    if (a.K < 1 || a.K > 64 || a.tt_cap_v != trim_tile_cap_v(a.K)) return hipErrorInvalidValue;
    if (a.tt_ntiles <= 0) return hipSuccess;
    switch ((a.K + 7) / 8) {
        case 1: return launch_trim_tile_l<1>(a, S, s);
        case 2: return launch_trim_tile_l<2>(a, S, s);
        case 3: return launch_trim_tile_l<3>(a, S, s);
        case 4: return launch_trim_tile_l<4>(a, S, s);
        case 5: return launch_trim_tile_l<5>(a, S, s);
        case 6: return launch_trim_tile_l<6>(a, S, s);
        case 7: return launch_trim_tile_l<7>(a, S, s);
        default: return launch_trim_tile_l<8>(a, S, s);
    }
}

hipError_t launch_trim(const TrimArgs &a, const double *S, hipStream_t s) {
    if (a.K < 1 || a.K > 64) return hipErrorInvalidValue;
    if (a.nv > 0)
        hipLaunchKernelGGL(k_zstar_h, dim3(static_cast<unsigned>((a.nv * a.K + 255) / 256)),
                           dim3(256), 0, s, a);
    switch ((a.K + 7) / 8) {
        case 1: launch_trim_layers<1>(a, S, s); break;
        case 2: launch_trim_layers<2>(a, S, s); break;
        case 3: launch_trim_layers<3>(a, S, s); break;
        case 4: launch_trim_layers<4>(a, S, s); break;
        case 5: launch_trim_layers<5>(a, S, s); break;
        case 6: launch_trim_layers<6>(a, S, s); break;
        case 7: launch_trim_layers<7>(a, S, s); break;
        default: launch_trim_layers<8>(a, S, s); break;
    }
    return hipGetLastError();
}

}  // namespace sesub
