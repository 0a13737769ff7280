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

}  // namespace
}  // namespace sesub
