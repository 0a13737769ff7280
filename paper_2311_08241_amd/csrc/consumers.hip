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
// wavefront per triangle / vertex, lane = layer: the sums over layers are wave
// reductions and the vertical recursion a suffix scan across lanes (so results
// equal the definition to rounding, not bit for bit); every load and store of
// layer data is one coalesced wave access.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double zstar_h(const TrimArgs &a, int64_t v, int k) {
    return a.h0[v * a.K + k] * ((a.H0[v] + a.eta_new[v]) / a.H0[v]);
}

__device__ __forceinline__ double wave_allsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Each wavefront handles EU elements at a time (independent load chains in flight).
// Workgroups are dealt round-robin to the XCDs; each owns a contiguous range.
constexpr int EU = 4;

__global__ void __launch_bounds__(256) k_trim(TrimArgs a) {
    const int lane = threadIdx.x & 63;
    const int K = a.K, k = lane;
    const bool act = k < K;
    // each workgroup owns a contiguous range of triangles (its vertices' layer data
    // then stays in one XCD's L2); its four wavefronts interleave over the range
    const int64_t chunk = (a.ne + gridDim.x - 1) / gridDim.x;
    const int64_t beg = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = min(a.ne, beg + chunk);
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    for (int64_t e0 = beg + wv; e0 < end; e0 += 4 * EU) {
        double hh[EU], ux[EU], uy[EU];
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            const int64_t e = e0 + u * 4;
            hh[u] = 0.0;
            ux[u] = 0.0;
            uy[u] = 0.0;
            if (act && e < end) {
                const int32_t *t = a.tri + 3 * e;
                const double ha = 0.5 * (a.hn[t[0] * (int64_t)K + k] + zstar_h(a, t[0], k));
                const double hb = 0.5 * (a.hn[t[1] * (int64_t)K + k] + zstar_h(a, t[1], k));
                const double hc = 0.5 * (a.hn[t[2] * (int64_t)K + k] + zstar_h(a, t[2], k));
                hh[u] = (ha + hb + hc) / 3.0;
                ux[u] = a.Ustar[(e * K + k) * 2];
                uy[u] = a.Ustar[(e * K + k) * 2 + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            const int64_t e = e0 + u * 4;
            if (e >= end) break;   // wave-uniform
            const double hs = wave_allsum(hh[u]);
            const double ex = wave_allsum(ux[u]) - a.Uavg[2 * e];
            const double ey = wave_allsum(uy[u]) - a.Uavg[2 * e + 1];
            if (act) {
                a.U[(e * K + k) * 2] = ux[u] - hh[u] / hs * ex;
                a.U[(e * K + k) * 2 + 1] = uy[u] - hh[u] / hs * ey;
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_zstar_w(TrimArgs a) {
    const int lane = threadIdx.x & 63;
    const int K = a.K, k = lane;
    const bool act = k < K;
    const int64_t chunk = (a.nv + gridDim.x - 1) / gridDim.x;
    const int64_t beg = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t end = min(a.nv, beg + chunk);
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    for (int64_t v0 = beg + wv; v0 < end; v0 += 4 * EU) {
        double t[EU];
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            const int64_t v = v0 + u * 4;
            t[u] = 0.0;
            if (act && v < end) {
                const double hnew = zstar_h(a, v, k);
                a.hnew[v * K + k] = hnew;
                double div = 0.0;
                const int32_t j1 = a.row_ptr[v + 1];
                for (int32_t j = a.row_ptr[v]; j < j1; ++j) {
                    const int32_t pcl = a.pcol[j];
                    const int64_t e = pcl / 3;
                    const int slot = pcl - 3 * (pcl / 3);
                    const double Ae = a.geom[4 * a.ne + e];
                    const double gbx = a.geom[e], gby = a.geom[a.ne + e],
                                 gcx = a.geom[2 * a.ne + e], gcy = a.geom[3 * a.ne + e];
                    const double Fx = a.U[(e * K + k) * 2], Fy = a.U[(e * K + k) * 2 + 1];
                    double pa, pb, pc;
                    slot_fluxes(Fx, Fy, gbx, gby, gcx, gcy, Ae, pa, pb, pc);
                    div += slot == 0 ? pa : (slot == 1 ? pb : pc);
                }
                t[u] = (hnew - a.hn[v * K + k]) / a.tau + div / a.Av[v] +
                       (k == 0 && a.W ? a.W[v] : 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            const int64_t v = v0 + u * 4;
            if (v >= end) break;   // wave-uniform
            // w[k] = -(t_k + t_{k+1} + ... + t_{K-1}): inclusive suffix scan across lanes
            double tt = t[u];
            for (int o = 1; o < 64; o <<= 1) {
                const double x = __shfl_down(tt, o, 64);
                if (lane + o < 64) tt += x;
            }
            double *w = a.w + v * (K + 1);
            if (act) w[k] = -tt;
            if (lane == 0) w[K] = 0.0;
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
__device__ __forceinline__ T visc_He(const ViscArgs &a, const T *H0, const T *eta, int32_t va,
                                     int32_t vb, int32_t vc) {
    if constexpr (F32) {
        const float h = (H0[va] + H0[vb] + H0[vc]) * (1.0f / 3.0f);
        if (a.linear_h) return h;
        return h + (static_cast<float>(a.eta_ref) + (eta[va] + eta[vb] + eta[vc]) * (1.0f / 3.0f));
    } else {
        if (a.linear_h) return (H0[va] + H0[vb] + H0[vc]) / 3.0;
        return ((H0[va] + eta[va]) + (H0[vb] + eta[vb]) + (H0[vc] + eta[vc])) / 3.0;
    }
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_visc_u(ViscArgs a) {
    using T2 = typename Vec2<T>::type;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.ne) return;
    const T *H0 = static_cast<const T *>(a.H0);
    const T *eta = static_cast<const T *>(a.eta);
    const int32_t *t = a.tri + 3 * e;
    const T He = visc_He<T, F32>(a, H0, eta, t[0], t[1], t[2]);
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
    T Hv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if constexpr (F32)
            Hv[k] = a.linear_h ? H0[t[k]] : H0[t[k]] + (eta[t[k]] + static_cast<float>(a.eta_ref));
        else
            Hv[k] = a.linear_h ? H0[t[k]] : H0[t[k]] + eta[t[k]];
    }
    const int32_t nbs[3] = {nb.x, nb.y, nb.z};
    T sx = 0, sy = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int32_t n = nbs[j];
        if (n < 0) continue;
        const T2 un = ub[n];
        const T Hj = static_cast<T>(0.5) * (Hv[j] + Hv[(j + 1) % 3]);
        const T dux = un.x - ue.x, duy = un.y - ue.y;
        const T A = A0 + Cv * vg[2 * j] * sqrt(dux * dux + duy * duy);
        const T c = Hj * A * vg[2 * j + 1];
        sx += c * dux;
        sy += c * duy;
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

hipError_t launch_trim(const TrimArgs &a, hipStream_t s) {
    // wavefronts loop over elements: at most 16 workgroups of 4 wavefronts per CU
    auto grid = [](int64_t n) {
        return static_cast<unsigned>(std::min<int64_t>((n + 4 * EU - 1) / (4 * EU), 256 * 16));
    };
    if (a.ne > 0) hipLaunchKernelGGL(k_trim, dim3(grid(a.ne)), dim3(256), 0, s, a);
    if (a.nv > 0) hipLaunchKernelGGL(k_zstar_w, dim3(grid(a.nv)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sesub
