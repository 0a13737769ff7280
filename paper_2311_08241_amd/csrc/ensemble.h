// Ensemble epilogue (gfx950): the volume rows of every member and the copy of final
// states that ended in the workspace, one launch each per call of the batched
// subcycle instead of one per member (Banerjee et al., arXiv 2311.08241: the FP64
// volume of Sec. 2.4 per member).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sesub {

// Ensemble: the volume rows of every member in one launch.  Member m's rows are
// blocks row0 .. row0 + rows - 1 (row0 ascending over members); row r sums width
// partials at part_off + r * width and writes add + sum to out[out_off + r].
struct VolMember {
    int64_t part_off, out_off;
    int32_t width, row0;
    double add;
};
hipError_t launch_vol_reduce_batch(const double *part, const VolMember *mem, int32_t nmem,
                                   int32_t rows, double *out, hipStream_t s);

// Ensemble: copy word ranges between two buffer pairs in one launch.  Range q covers
// words [start, start + (cum_{q+1} - cum_q)) of pair `pair` (0: src0 -> dst0, 1: src1
// -> dst1), at the same offset in source and destination; cum ascending, cum_0 = 0.
struct CopyRange {
    int64_t start, cum;
    int32_t pair, pad;
};
hipError_t launch_copy_ranges(const uint32_t *src0, uint32_t *dst0, const uint32_t *src1,
                              uint32_t *dst1, const CopyRange *r, int32_t nr, int64_t total,
                              hipStream_t s);

}  // namespace sesub
