// Nearest neighbours in descriptor space, both directions (Algorithm 1's
// pre-matching cache, extended to the reciprocal test).  Every fragment's rows
// query its partner fragment: D(i,j) = sum_c (F_i[c] - G_j[c])^2 in float32,
// always accumulated in the same order (d2_row), argmin over valid rows with
// ties to the lowest index.
//
// LSR_FP32 scans every candidate on the vector ALUs.
// LSR_BF16_SCREEN (match_bf16.hip) screens on the matrix cores, re-ranks the
// surviving candidates with d2_row and falls back to the scan for rows it
// cannot certify, so both modes return identical bits.
#include <algorithm>

#include "match_common.h"

namespace lsr {

constexpr int MT = 256;         // threads per block
constexpr int MR = 2;           // query rows per thread
constexpr int MC = 64;          // candidates staged per LDS round
constexpr int MS = 36;          // LDS row stride (floats), 33 rounded up for 16-byte reads

// Block (x, y): 512 query rows of one fragment (2 per thread, held in
// registers) against candidate range y of SPLIT ranges of the partner
// (candidates staged in LDS 64 at a time, read by every thread at once).
// A range's best per row is merged into key[row] = min((distance bits << 32)
// | index) with a 64-bit atomic minimum: distances are non-negative, so the
// bits order like the values, and equal distances keep the lowest index, as
// a single scan in index order would.  One split (a batch of many pairs)
// fills the chip with query blocks alone; a single pair needs several.
__global__ void __launch_bounds__(MT) k_match_fp32(const Frag *frag, const Blk *blk, const float *F,
                                                   const int32_t *valid, int split, unsigned long long *key) {
    __shared__ __align__(16) float cand[MC * MS];
    __shared__ int32_t cval[MC];
    const Blk b = blk[blockIdx.x];
    const Frag &Fq = frag[b.frag];
    if (Fq.partner < 0) return;
    const Frag &Fc = frag[Fq.partner];
    const int per = ((Fc.n + split - 1) / split + MC - 1) / MC * MC;
    const int j_lo = (int)blockIdx.y * per, j_hi = min(Fc.n, j_lo + per);
    if (j_lo >= j_hi) return;
    float q[MR][MS];
    bool qv[MR];
    float best[MR];
    int32_t bj[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
        int i = b.start + threadIdx.x + r * MT;
        qv[r] = i < Fq.n && valid[Fq.off + i];
        const float *src = F + (Fq.off + (qv[r] ? i : 0)) * FD;
#pragma unroll
        for (int c = 0; c < MS; ++c) q[r][c] = (qv[r] && c < FD) ? src[c] : 0.f;
        best[r] = INFINITY;
        bj[r] = -1;
    }
    for (int c0 = j_lo; c0 < j_hi; c0 += MC) {
        __syncthreads();
        const float *base = F + (Fc.off + c0) * FD;
        int lim = min(MC, j_hi - c0);
        for (int t = threadIdx.x; t < MC * MS; t += MT) {
            int jj = t / MS, c = t - jj * MS;
            cand[t] = (jj < lim && c < FD) ? base[jj * FD + c] : 0.f;
        }
        if (threadIdx.x < MC) cval[threadIdx.x] = threadIdx.x < lim ? valid[Fc.off + c0 + threadIdx.x] : 0;
        __syncthreads();
        for (int jj = 0; jj < lim; ++jj) {
            if (!cval[jj]) continue;
            const float *x = cand + jj * MS;
#pragma unroll
            for (int r = 0; r < MR; ++r) {
                float d = d2_row(q[r], x);
                if (d < best[r]) { best[r] = d; bj[r] = c0 + jj; }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < MR; ++r) {
        int i = b.start + threadIdx.x + r * MT;
        if (i < Fq.n && qv[r] && bj[r] >= 0)
            atomicMin(&key[Fq.off + i], ((unsigned long long)__float_as_uint(best[r]) << 32) | (uint32_t)bj[r]);
    }
}

__global__ void __launch_bounds__(256) k_match_fp32_out(const Frag *frag, const Blk *blk, const int32_t *valid,
                                                        const unsigned long long *key, int32_t *nn, float *dist) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fq = frag[b.frag];
    const int i = b.start + threadIdx.x;
    if (i >= Fq.n) return;
    const int64_t gi = Fq.off + i;
    const unsigned long long k = key[gi];
    const bool found = Fq.partner >= 0 && valid[gi] && k != ~0ull;
    nn[gi] = found ? (int32_t)(uint32_t)k : -1;
    dist[gi] = found ? __uint_as_float((uint32_t)(k >> 32)) : INFINITY;
}

// One block per listed row: threads split the candidates, then the block
// takes the minimum (value, then index).  Used for rows the screen could not
// certify; *count rows are listed (device), the grid is an upper bound.
__global__ void __launch_bounds__(256) k_match_rows(const Frag *frag, const float *F, const int32_t *valid,
                                                    const int32_t *rows, const int32_t *row_frag, const int32_t *count,
                                                    int32_t *nn, float *dist) {
    __shared__ float sv[256];
    __shared__ int32_t si[256];
    if ((int)blockIdx.x >= *count) return;
    const int32_t f = row_frag[blockIdx.x];
    const Frag &Fq = frag[f];
    const Frag &Fc = frag[Fq.partner];
    const int32_t i = rows[blockIdx.x];
    float q[MS];
    const float *src = F + (Fq.off + i) * FD;
#pragma unroll
    for (int c = 0; c < MS; ++c) q[c] = c < FD ? src[c] : 0.f;
    float best = INFINITY;
    int32_t bj = -1;
    float x[MS];
    for (int j = threadIdx.x; j < Fc.n; j += 256) {
        if (!valid[Fc.off + j]) continue;
        const float *cr = F + (Fc.off + j) * FD;
#pragma unroll
        for (int c = 0; c < MS; ++c) x[c] = c < FD ? cr[c] : 0.f;
        float d = d2_row(q, x);
        if (d < best) { best = d; bj = j; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bj;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            float v2 = sv[threadIdx.x + o];
            int32_t j2 = si[threadIdx.x + o];
            float v1 = sv[threadIdx.x];
            int32_t j1 = si[threadIdx.x];
            bool take = (v2 < v1) || (v2 == v1 && j2 >= 0 && (j1 < 0 || j2 < j1));
            if (take) { sv[threadIdx.x] = v2; si[threadIdx.x] = j2; }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        nn[Fq.off + i] = si[0];
        dist[Fq.off + i] = sv[0];
    }
}

hipError_t launch_match_fp32(const GridBufs &g, const DescBufs &d, MatchBufs &m, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipError_t e = fill<unsigned long long>(m.nnkey, ~0ull, g.ntot, s);
    if (e != hipSuccess) return e;
    // candidate ranges per query block: enough blocks for 8 per CU
    const int split = std::max(1, std::min(64, 2048 / std::max(1, g.nblk512)));
    if (g.nblk512 > 0)
        hipLaunchKernelGGL(k_match_fp32, dim3(g.nblk512, split), dim3(MT), 0, s, (const Frag *)g.frag,
                           (const Blk *)g.blk512, (const float *)d.F, (const int32_t *)d.valid, split, m.nnkey);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_match_fp32_out, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)d.valid, (const unsigned long long *)m.nnkey, m.nn, m.dist);
    return hipGetLastError();
}

hipError_t launch_match_rows(const GridBufs &g, const DescBufs &d, const int32_t *rows, const int32_t *row_frag,
                             const int32_t *count, int64_t max_rows, MatchBufs &m, hipStream_t s) {
    if (max_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_match_rows, dim3((unsigned)max_rows), dim3(256), 0, s, (const Frag *)g.frag,
                       (const float *)d.F, (const int32_t *)d.valid, rows, row_frag, count, m.nn, m.dist);
    return hipGetLastError();
}

}  // namespace lsr
