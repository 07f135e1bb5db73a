// Descriptor distance shared by every matching kernel, so that the scan, the
// re-rank and the fallback produce bit-identical float32 distances.
#pragma once
#include "lsr_internal.h"

namespace lsr {

// sum_{c<33} (q_c - x_c)^2, one fixed order of float32 operations.
__device__ __forceinline__ float d2_row(const float *q, const float *x) {
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < FD; ++c) {
        float t = __fsub_rn(q[c], x[c]);
        acc = __fmaf_rn(t, t, acc);
    }
    return acc;
}

hipError_t launch_match_fp32(const GridBufs &g, const DescBufs &d, MatchBufs &m, hipStream_t s);
hipError_t launch_match_rows(const GridBufs &g, const DescBufs &d, const int32_t *rows, const int32_t *row_frag,
                             const int32_t *count, int64_t max_rows, MatchBufs &m, hipStream_t s);

}  // namespace lsr
