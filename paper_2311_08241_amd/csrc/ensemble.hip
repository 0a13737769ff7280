// Ensemble epilogue kernels (gfx950, wave64); see ensemble.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "ensemble.h"

namespace sesub {

namespace {

// Same thread partition and tree as k_vol_reduce, so each member's rows equal a
// standalone reduction bit for bit.
__global__ void __launch_bounds__(256) k_vol_reduce_batch(const double *part,
                                                          const VolMember *mem, int32_t nmem,
                                                          double *out) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    int lo = 0, hi = nmem - 1;   // last member with row0 <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mem[mid].row0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const VolMember m = mem[lo];
    const int64_t r = b - m.row0;
    const double *row = part + m.part_off + r * m.width;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m.width; i += 256) s += row[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[m.out_off + r] = m.add + ((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ void __launch_bounds__(256) k_copy_ranges(const uint32_t *src0, uint32_t *dst0,
                                                     const uint32_t *src1, uint32_t *dst1,
                                                     const CopyRange *rg, int32_t nr,
                                                     int64_t total) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < total;
         j += stride) {
        int lo = 0, hi = nr - 1;   // last range with cum <= j
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rg[mid].cum <= j) lo = mid;
            else hi = mid - 1;
        }
        const int64_t w = rg[lo].start + (j - rg[lo].cum);
        if (rg[lo].pair == 0) dst0[w] = src0[w];
        else dst1[w] = src1[w];
    }
}

}  // namespace

hipError_t launch_vol_reduce_batch(const double *part, const VolMember *mem, int32_t nmem,
                                   int32_t rows, double *out, hipStream_t s) {
    if (rows <= 0 || nmem <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vol_reduce_batch, dim3(rows), dim3(256), 0, s, part, mem, nmem, out);
    return hipGetLastError();
}

hipError_t launch_copy_ranges(const uint32_t *src0, uint32_t *dst0, const uint32_t *src1,
                              uint32_t *dst1, const CopyRange *r, int32_t nr, int64_t total,
                              hipStream_t s) {
    if (total <= 0 || nr <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 256 * 32);
    hipLaunchKernelGGL(k_copy_ranges, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, src0,
                       dst0, src1, dst1, r, nr, total);
    return hipGetLastError();
}

}  // namespace sesub
