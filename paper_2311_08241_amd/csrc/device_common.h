// Device helpers shared by the subcycle kernels (kernels.hip) and the consumer
// kernels of the averaged transport and forcing (consumers.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sesub {
namespace {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// A double moved between lanes by one DPP control (both halves; rows outside ROWMASK
// receive 0).
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWMASK, 0xf,
                                               false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

// Sum over the wavefront (every lane active) in a fixed order without LDS: within each
// row of 16 lanes by quad permutations and mirrors, then row 0 into row 1 and row 2
// into row 3 (broadcast of lane 15), then rows 0-1 into row 3 (broadcast of lane 31).
// The total is in lane 63.
__device__ __forceinline__ double wave_sum_last(double v) {
    v += dpp_f64<0xB1>(v);          // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);          // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);         // row_half_mirror
    v += dpp_f64<0x140>(v);         // row_mirror
    v += dpp_f64<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ void set_fault(uint32_t *faults, uint32_t bit) {
    atomicOr(faults, bit);
}

template <typename T> __device__ __forceinline__ bool finite_val(T v) { return isfinite(v); }

// Sub-cell fluxes F . S_k of a transport F through the median-dual boundary
// pieces of the triangle's three vertices, S_k = -A_e grad N_k (FP64, the
// operation order of the CPU definition).
__device__ __forceinline__ void slot_fluxes(double Fx, double Fy, double gbx, double gby,
                                            double gcx, double gcy, double Ae, double &pa,
                                            double &pb, double &pc) {
    const double gax = -(gbx + gcx), gay = -(gby + gcy);
    pa = Fx * (-Ae * gax) + Fy * (-Ae * gay);
    pb = Fx * (-Ae * gbx) + Fy * (-Ae * gby);
    pc = Fx * (-Ae * gcx) + Fy * (-Ae * gcy);
}


// Barotropic viscous term (eq. (eq:viscosity_BT)), shared by the plain kernels and the
// tile kernel so that both evaluate the same operations in the same order.
// Triangle depth H_e: mean of H0 + eta at its vertices (mean H0 with linear_h); FP32
// eta holds eta - eta_ref.
template <typename T, bool F32>
__device__ __forceinline__ T visc_tri_depth(bool linear_h, float eta_ref, T h0a, T h0b, T h0c,
                                            T ea, T eb, T ec) {
    if constexpr (F32) {
        const float h = (h0a + h0b + h0c) * (1.0f / 3.0f);
        if (linear_h) return h;
        return h + (eta_ref + (ea + eb + ec) * (1.0f / 3.0f));
    } else {
        if (linear_h) return (h0a + h0b + h0c) / 3.0;
        return ((h0a + ea) + (h0b + eb) + (h0c + ec)) / 3.0;
    }
}

// Depth H0 + eta at a vertex (H0 with linear_h).
template <typename T, bool F32>
__device__ __forceinline__ T visc_vtx_depth(bool linear_h, float eta_ref, T h0, T e) {
    if (linear_h) return h0;
    if constexpr (F32)
        return h0 + (e + eta_ref);
    else
        return h0 + e;
}

// Two-point flux through one edge: coefficient A = A0 + Cv l |du|, flux
// H_j A (l/d) du added to (sx, sy).
template <typename T>
__device__ __forceinline__ void visc_edge(T A0, T Cv, T Hj, T l, T lod, T dux, T duy, T &sx,
                                          T &sy) {
    const T A = A0 + Cv * l * sqrt(dux * dux + duy * duy);
    const T c = Hj * A * lod;
    sx += c * dux;
    sy += c * duy;
}

}  // namespace
}  // namespace sesub
