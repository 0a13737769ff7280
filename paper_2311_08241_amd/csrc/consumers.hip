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
// ascending triangle order, and the diasurface velocity from the bottom up.
//   k_zstar_h       h^{n+1} = h0 (H0 + eta) / H0, one thread per vertex-layer; also
//                   hn + h^{n+1}, parked in w until k_zstar_w overwrites it
//   k_trim          one wavefront per EU consecutive triangles, lane = layer:
//                   6 x the mid thickness (the common factor cancels in the trim
//                   weights), layer sums by lane shuffles, trimmed transports
//   k_zstar_w       one wavefront per vertex, lane = layer: the CSR row's fluxes
//                   AB triangles at a time (all loads of a batch in flight), then
//                   w by a suffix scan across lanes
// Indices a wavefront needs (triangle vertices, CSR columns) are loaded by its
// lanes in one access and broadcast with readlane, so no scalar-load chain sits
// between an element and its layer data.  Results equal the definition to rounding
// (tree sums, reciprocals), not bit for bit.
// ---------------------------------------------------------------------------
// Rotation right by n lanes within each row of 16 (DPP row_ror), on an FP64 value.
template <int N> __device__ __forceinline__ double row_ror(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0x120 + N, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x120 + N, 0xf, 0xf,
                                               false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Sum over the 64 lanes, returned to every lane: rotations within each row of 16,
// then the four row sums.
__device__ __forceinline__ double wave_allsum(double v) {
    v += row_ror<8>(v);
    v += row_ror<4>(v);
    v += row_ror<2>(v);
    v += row_ror<1>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ __forceinline__ int32_t bcast(int32_t v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}

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

// wave-level contiguous range of n elements
__device__ __forceinline__ void wave_range(int64_t n, int64_t &beg, int64_t &end) {
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    const int64_t gw = xcd_block() * (blockDim.x >> 6) +
                       __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t chunk = (n + nw - 1) / nw;
    beg = gw * chunk;
    end = min(n, beg + chunk);
}

constexpr int EU = 4;   // triangles per wavefront iteration of k_trim

__global__ void __launch_bounds__(256) k_trim(TrimArgs a) {
    const int lane = threadIdx.x & 63;
    const int K = a.K, k = lane;
    const bool act = k < K;
    int64_t beg, end;
    wave_range(a.ne, beg, end);
    if (beg >= end) return;
    // triangle indices of an iteration, one per lane (lane 3u + c: vertex c of e0 + u),
    // loaded one iteration ahead
    int32_t myt = a.tri[3 * beg + min<int64_t>(lane, 3 * (end - beg) - 1)];
    for (int64_t e0 = beg; e0 < end; e0 += EU) {
        const int nu = static_cast<int>(min<int64_t>(EU, end - e0));
        double hh[EU], ux[EU], uy[EU];
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            const int uu = min(u, nu - 1);   // past the range: repeat the last triangle
            const int64_t ta = bcast(myt, 3 * uu), tb = bcast(myt, 3 * uu + 1),
                          tc = bcast(myt, 3 * uu + 2);
            hh[u] = 0.0;
            ux[u] = 0.0;
            uy[u] = 0.0;
            if (act) {
                const double *hm = a.w;   // hn + hnew, row stride K + 1
                hh[u] = (hm[ta * (K + 1) + k] + hm[tb * (K + 1) + k]) + hm[tc * (K + 1) + k];
                const double2 us = reinterpret_cast<const double2 *>(a.Ustar)[(e0 + uu) * K + k];
                ux[u] = us.x;
                uy[u] = us.y;
            }
        }
        const int64_t e1 = e0 + EU;
        if (e1 < end) myt = a.tri[3 * e1 + min<int64_t>(lane, 3 * (end - e1) - 1)];
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            if (u >= nu) break;   // wave-uniform
            const int64_t e = e0 + u;
            const double hs = wave_allsum(hh[u]);
            const double ex = wave_allsum(ux[u]) - a.Uavg[2 * e];
            const double ey = wave_allsum(uy[u]) - a.Uavg[2 * e + 1];
            const double q = hh[u] * (1.0 / hs);
            if (act) {
                double2 r;
                r.x = ux[u] - q * ex;
                r.y = uy[u] - q * ey;
                reinterpret_cast<double2 *>(a.U)[e * K + k] = r;
            }
        }
    }
}

// k_zstar_w: VU consecutive vertices per wavefront iteration (their CSR rows inside one
// 64-column window), AB triangles of each row per batch of loads; other groups take
// the one-vertex form.
constexpr int ZW_VU = 2, ZW_AB = 6;

template <int VU, int AB>
__global__ void __launch_bounds__(256) k_zstar_w(TrimArgs a, const double *S) {
    const int lane = threadIdx.x & 63;
    const int K = a.K, k = lane;
    const bool act = k < K;
    const double inv_tau = 1.0 / a.tau;
    // read-only table indexed by wave-uniform values: scalar loads
    const __attribute__((address_space(4))) double *S4 =
        (const __attribute__((address_space(4))) double *)(S);
    const double2 *U2 = reinterpret_cast<const double2 *>(a.U);
    // flux of the trimmed transport of CSR entry pcl = 3 e + slot through the slot's
    // sub-cell boundary, layer k
    auto flux = [&](int32_t pcl) {
        const int64_t e = pcl / 3;
        const double svx = S4[2 * pcl], svy = S4[2 * pcl + 1];
        const double2 F = act ? U2[e * K + k] : make_double2(0.0, 0.0);
        return F.x * svx + F.y * svy;
    };
    // w[k] = -(t_k + t_{k+1} + ... + t_{K-1}): inclusive suffix scan across lanes
    auto finish = [&](int64_t v, double hnew, double hn, double div) {
        double t = (hnew - hn) * inv_tau + div * (1.0 / a.Av[v]) +
                   (k == 0 && a.W ? a.W[v] : 0.0);
        if (!act) t = 0.0;
        for (int o = 1; o < 64; o <<= 1) {
            const double x = __shfl_down(t, o, 64);
            if (lane + o < 64) t += x;
        }
        double *w = a.w + v * (K + 1);
        if (act) w[k] = -t;
        if (lane == 0) w[K] = 0.0;
    };
    int64_t beg, end;
    wave_range(a.nv, beg, end);
    for (int64_t vb = beg; vb < end; vb += 63) {
        // row bounds of up to 63 vertices: lane u holds row_ptr[vb + u]
        const int nvb = static_cast<int>(min<int64_t>(63, end - vb));
        const int32_t rp = a.row_ptr[vb + min(lane, nvb)];
        const int32_t jend = bcast(rp, nvb);
        // CSR columns, 64 at a time: lane i holds pcol[cbase + i]; cbase only moves
        // forward, so it never passes the start of a later row
        int32_t cbase = bcast(rp, 0);
        int32_t pc = a.pcol[min(cbase + lane, jend - 1)];
        for (int u0 = 0; u0 < nvb; u0 += VU) {
            const int nu = min(VU, nvb - u0);
            const int32_t jf = bcast(rp, u0), jl = bcast(rp, u0 + nu);
            if (nu == VU && jl - jf <= 64) {
                if (jl > cbase + 64) {
                    cbase = jf;
                    pc = a.pcol[min(cbase + lane, jend - 1)];
                }
                int32_t j0[VU], len[VU];
                double hnew[VU], hn[VU], div[VU];
                int maxlen = 0;
#pragma unroll
                for (int u = 0; u < VU; ++u) {
                    const int64_t v = vb + u0 + u;
                    j0[u] = bcast(rp, u0 + u);
                    len[u] = bcast(rp, u0 + u + 1) - j0[u];   // >= 1: every vertex has a triangle
                    maxlen = max(maxlen, len[u]);
                    hnew[u] = act ? a.hnew[v * K + k] : 0.0;
                    hn[u] = act ? a.hn[v * K + k] : 0.0;
                    div[u] = 0.0;
                }
                for (int off = 0; off < maxlen; off += AB) {
                    double fl[VU][AB];
#pragma unroll
                    for (int u = 0; u < VU; ++u)
#pragma unroll
                        for (int q = 0; q < AB; ++q)   // past a row's end: its last entry again
                            fl[u][q] = flux(bcast(pc, j0[u] + min(off + q, len[u] - 1) - cbase));
#pragma unroll
                    for (int u = 0; u < VU; ++u)
#pragma unroll
                        for (int q = 0; q < AB; ++q)
                            if (off + q < len[u]) div[u] += fl[u][q];
                }
#pragma unroll
                for (int u = 0; u < VU; ++u) finish(vb + u0 + u, hnew[u], hn[u], div[u]);
                continue;
            }
            for (int u = u0; u < u0 + nu; ++u) {
                const int64_t v = vb + u;
                const int32_t j0 = bcast(rp, u), j1 = bcast(rp, u + 1);
                const double hnew = act ? a.hnew[v * K + k] : 0.0;
                const double hn = act ? a.hn[v * K + k] : 0.0;
                double div = 0.0;
                for (int32_t j = j0; j < j1; j += AB) {
                    // this batch's columns j .. min(j + AB, j1) - 1 inside the window
                    // [cbase, cbase + 64) (wave-uniform; rows of any length)
                    if (min(j + AB, j1) > cbase + 64) {
                        cbase = j;
                        pc = a.pcol[min(cbase + lane, jend - 1)];
                    }
                    double fl[AB];
#pragma unroll
                    for (int q = 0; q < AB; ++q) fl[q] = flux(bcast(pc, min(j + q, j1 - 1) - cbase));
#pragma unroll
                    for (int q = 0; q < AB; ++q)
                        if (j + q < j1) div += fl[q];
                }
                finish(v, hnew, hn, div);
            }
        }
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

hipError_t launch_trim(const TrimArgs &a, const double *S, hipStream_t s) {
    // wavefronts loop over contiguous ranges; up to 64 workgroups of 4 per CU (more than
    // fit at once: short ranges balance the tail)
    if (a.nv > 0)
        hipLaunchKernelGGL(k_zstar_h, dim3(static_cast<unsigned>((a.nv * a.K + 255) / 256)),
                           dim3(256), 0, s, a);
    if (a.ne > 0)
        hipLaunchKernelGGL(k_trim, dim3(static_cast<unsigned>(std::min<int64_t>(
                                        (a.ne + 4 * EU - 1) / (4 * EU), 256 * 64))),
                           dim3(256), 0, s, a);
    if (a.nv > 0)
        hipLaunchKernelGGL((k_zstar_w<ZW_VU, ZW_AB>),
                           dim3(static_cast<unsigned>(std::min<int64_t>((a.nv + 63) / 64, 256 * 64))),
                           dim3(256), 0, s, a, S);
    return hipGetLastError();
}

}  // namespace sesub
