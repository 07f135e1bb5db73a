// Reciprocal test, quadruple consistency filter and compaction.
//
// Reciprocal: (i, nnQ(i)) is kept when nnP(nnQ(i)) = i.
// Consistency (Algorithm 1's pre-rejection, used as a filter): the reciprocal
// correspondences C of a pair are packed in ascending P index; trial t draws
// four distinct members of C, slot s taking the first of up to 64 draws
// c = ((r >> 32) * |C|) >> 32 that differs from the earlier slots, with r the
// n-th output of SplitMix64 (Steele, Lea and Flood 2014) for the given seed
// and n = (t << 8) | (s << 6) | attempt.  The closed quadrilateral passes when
// every edge length ratio lies within tau in both directions (squared, FP64);
// the correspondences of a passing trial are flagged.
// Compaction: flagged correspondences in ascending P index, as float xyz of p
// and q, the input of the pose solve.
#include <algorithm>

#include "lsr_internal.h"

namespace lsr {

__global__ void __launch_bounds__(256) k_mutual(const Frag *frag, const Blk *blk, const int32_t *nn, uint8_t *mutual,
                                                PairState *ps) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    bool m = false;
    if (i < F.n && F.partner >= 0) {
        const Frag &G = frag[F.partner];
        int32_t j = nn[F.off + i];
        m = j >= 0 && nn[G.off + j] == i;
        mutual[F.off + i] = m ? 1 : 0;
    }
    unsigned long long bal = __ballot(m);
    const int w = threadIdx.x >> 6;
    __shared__ int cnt[4];
    if ((threadIdx.x & 63) == 0) cnt[w] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0 && ps && F.pair >= 0 && (b.frag & 1) == 0) {
        int t = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        if (t) atomicAdd(&ps[F.pair].n_recip, (unsigned long long)t);
    }
}

hipError_t launch_mutual(const GridBufs &g, MatchBufs &m, PairState *ps, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mutual, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)m.nn, m.mutual, ps);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea and Flood 2014): the n-th output for a seed is the
// finaliser applied to the state seed + (n + 1) * golden-gamma.  Consecutive
// draws of one slot only add the gamma to the state; only the upper 32 bits
// of the output are used (the index draw below).
constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint32_t splitmix64_hi(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

constexpr int TPB = 8192;    // trials per block (the trial table's granularity)
constexpr int CONS_THREADS[] = {256, 128, 512};   // block widths the autotuner picks from
constexpr int N_CONS_SHAPES = sizeof(CONS_THREADS) / sizeof(CONS_THREADS[0]);

// usable[g] = 1 for a P point with a reciprocal correspondence inside Q (scan input).
__global__ void __launch_bounds__(256) k_corr_usable(const Frag *frag, const Blk *blk, const int32_t *nn,
                                                     const uint8_t *mutual, int32_t *usable) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= P.n) return;
    bool u = false;
    if ((b.frag & 1) == 0 && P.partner >= 0 && mutual[P.off + i]) {
        int32_t j = nn[P.off + i];
        u = j >= 0 && j < frag[P.partner].n;
    }
    usable[P.off + i] = u ? 1 : 0;
}

// C packed in ascending P index at the scanned slots, one trial slot reading 32
// contiguous bytes: (p_i, q_nnQ(i)) and i; the pair's list start and length.
__global__ void __launch_bounds__(256) k_corr_pack(const Frag *frag, const Blk *blk, const int32_t *nn,
                                                   const int32_t *usable, const int32_t *cpos, float4 *cpack,
                                                   PairState *ps) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    if ((b.frag & 1) || P.partner < 0) return;
    const Frag &Q = frag[P.partner];
    int i = b.start + threadIdx.x;
    if (i >= P.n) return;
    const int64_t gi = P.off + i;
    if (i == P.n - 1) {
        ps[P.pair].c_off = cpos[P.off];
        ps[P.pair].c_cnt = cpos[gi] + usable[gi] - cpos[P.off];
    }
    if (!usable[gi]) return;
    const int32_t j = nn[gi];
    const int64_t c = cpos[gi];
    cpack[2 * c] = make_float4(P.src[0][i], P.src[1][i], P.src[2][i], Q.src[0][j]);
    cpack[2 * c + 1] = make_float4(Q.src[1][j], Q.src[2][j], __int_as_float(i), 0.f);
}

// Edge test of one drawn quadruple (positions in the pair's packed C); flags
// the correspondences' P points when it passes.  The edges are tested in
// order and a correspondence is fetched only while every edge so far holds:
// the verdict is that of the full test, with fewer random gathers (the
// kernel is bound by them).
__device__ __forceinline__ bool edge_ok(const float4 &a0, const float4 &a1, const float4 &b0, const float4 &b1,
                                        double t2) {
    double a = pdist2(a0.x, a0.y, a0.z, b0.x, b0.y, b0.z);
    double c = pdist2(a0.w, a1.x, a1.y, b0.w, b1.x, b1.y);
    return !(a == 0.0 || c == 0.0 || a < t2 * c || c < t2 * a);
}

__device__ __forceinline__ int quad_test(const float4 *cp, int4 e, double t2, int32_t *flag) {
    const float4 p0 = cp[2 * e.x], p1 = cp[2 * e.y], q0 = cp[2 * e.x + 1], q1 = cp[2 * e.y + 1];
    if (!edge_ok(p0, q0, p1, q1, t2)) return 0;
    const float4 p2 = cp[2 * e.z], q2 = cp[2 * e.z + 1];
    if (!edge_ok(p1, q1, p2, q2, t2)) return 0;
    const float4 p3 = cp[2 * e.w], q3 = cp[2 * e.w + 1];
    if (!edge_ok(p2, q2, p3, q3, t2) || !edge_ok(p3, q3, p0, q0, t2)) return 0;
    flag[__float_as_int(q0.z)] = 1;
    flag[__float_as_int(q1.z)] = 1;
    flag[__float_as_int(q2.z)] = 1;
    flag[__float_as_int(q3.z)] = 1;
    return 1;
}

// Index drawn from SplitMix64 state z: a position in C.
__device__ __forceinline__ int draw(uint64_t z, uint32_t nC) {
    return (int)(((uint64_t)splitmix64_hi(z) * nC) >> 32);
}

// A slot's member: the first of up to 64 draws from state z on (attempts
// advance the state by one gamma) that differs from x, y and w (the earlier
// slots, repeated when there are fewer); -1 when all 64 repeat one of them.
__device__ int slot_member(uint64_t z, uint32_t nC, int x, int y, int w) {
    for (int a = 0; a < 64; ++a, z += GAMMA) {
        const int i = draw(z, nC);
        if (i != x && i != y && i != w) return i;
    }
    return -1;
}

// Each thread takes trials first + threadIdx.x + k CT of its block.  A trial
// whose four slots' first draws are pairwise distinct keeps them (each slot
// accepts its first draw, which already differs from the earlier slots); with
// |C| in the thousands that is nearly every trial, so the common case is four
// hashes and the edge test in straight-line code.  A trial with a repeat
// takes its slots again in order with further attempts, as defined above.
// Fewer than four members in C: no trial can draw a quadruple.
template <int CT>
__global__ void __launch_bounds__(CT) k_consistency(const Frag *frag, const TrialBlk *tb, const float4 *cpack,
                                                    int32_t *flag, double t2, uint64_t seed, PairState *ps) {
    const TrialBlk b = tb[blockIdx.x];
    const Frag &P = frag[2 * b.pair];
    const uint32_t nC = (uint32_t)ps[b.pair].c_cnt;
    const float4 *cp = cpack + 2 * ps[b.pair].c_off;
    int32_t *fl = flag + P.off;
    const int64_t end = nC >= 4 ? min(b.count, b.first + TPB) : b.first;
    int passed = 0;
    for (int64_t t = b.first + threadIdx.x; t < end; t += CT) {
        const uint64_t z0 = seed + (((uint64_t)t << 8) + 1ull) * GAMMA;      // slot 0, attempt 0
        const uint64_t z1 = z0 + 64ull * GAMMA, z2 = z0 + 128ull * GAMMA, z3 = z0 + 192ull * GAMMA;
        const int i0 = draw(z0, nC);
        int i1 = draw(z1, nC), i2 = draw(z2, nC), i3 = draw(z3, nC);
        const bool rep = (i1 == i0) | (i2 == i0) | (i2 == i1) | (i3 == i0) | (i3 == i1) | (i3 == i2);
        if (rep) {
            i1 = slot_member(z1, nC, i0, i0, i0);
            i2 = i1 < 0 ? -1 : slot_member(z2, nC, i0, i1, i1);
            i3 = i2 < 0 ? -1 : slot_member(z3, nC, i0, i1, i2);
        }
        if (i3 >= 0) passed += quad_test(cp, make_int4(i0, i1, i2, i3), t2, fl);
    }
    // passing-trial count per pair (integer, order independent)
    for (int o = 32; o > 0; o >>= 1) passed += __shfl_xor(passed, o, 64);
    if ((threadIdx.x & 63) == 0 && passed) atomicAdd(&ps[b.pair].trials_passed, (unsigned long long)passed);
}

hipError_t launch_consistency(const GridBufs &g, MatchBufs &m, PairState *ps, const TrialBlk *tb, int ntb,
                              float tau, uint64_t seed, int shape, int32_t *scan_tmp, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_corr_usable, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)m.nn, (const uint8_t *)m.mutual, m.flag);
    hipError_t e = exclusive_scan_i32(m.flag, m.kpos, g.ntot, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_corr_pack, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)m.nn, (const int32_t *)m.flag, (const int32_t *)m.kpos, m.cpack, ps);
    if ((e = fill<int32_t>(m.flag, 0, g.ntot, s)) != hipSuccess || ntb == 0) return e;
    double t2 = (double)tau * (double)tau;
    const Frag *fr = (const Frag *)g.frag;
    const float4 *cp = (const float4 *)m.cpack;
    switch (shape) {
    case 0: hipLaunchKernelGGL(k_consistency<CONS_THREADS[0]>, dim3(ntb), dim3(CONS_THREADS[0]), 0, s, fr, tb, cp,
                               m.flag, t2, seed, ps); break;
    case 1: hipLaunchKernelGGL(k_consistency<CONS_THREADS[1]>, dim3(ntb), dim3(CONS_THREADS[1]), 0, s, fr, tb, cp,
                               m.flag, t2, seed, ps); break;
    case 2: hipLaunchKernelGGL(k_consistency<CONS_THREADS[2]>, dim3(ntb), dim3(CONS_THREADS[2]), 0, s, fr, tb, cp,
                               m.flag, t2, seed, ps); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int trials_per_block() { return TPB; }
int consistency_shapes() { return N_CONS_SHAPES; }

// Flagged correspondences, in ascending P index, gathered into compact xyz
// arrays; per pair the list starts at kpos[P.off].
__global__ void __launch_bounds__(256) k_compact(const Frag *frag, const Blk *blk, const int32_t *flag,
                                                 const int32_t *kpos, const int32_t *nn, float *kp, float *kq,
                                                 int32_t *ki, PairState *ps) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    if ((b.frag & 1) || P.partner < 0) return;          // P fragments only
    const Frag &Q = frag[P.partner];
    int i = b.start + threadIdx.x;
    bool f = i < P.n && flag[P.off + i];
    if (f) {
        int64_t pos = kpos[P.off + i];
        int32_t j = nn[P.off + i];
        kp[3 * pos] = P.src[0][i]; kp[3 * pos + 1] = P.src[1][i]; kp[3 * pos + 2] = P.src[2][i];
        kq[3 * pos] = Q.src[0][j]; kq[3 * pos + 1] = Q.src[1][j]; kq[3 * pos + 2] = Q.src[2][j];
        ki[pos] = i;
    }
    if (b.start == 0 && threadIdx.x == 0 && ps && P.pair >= 0) ps[P.pair].k_off = kpos[P.off];
    unsigned long long bal = __ballot(f);
    __shared__ int cnt[4];
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0 && ps && P.pair >= 0) {
        int t = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        if (t) atomicAdd(&ps[P.pair].n_consistent, (unsigned long long)t);
    }
}

hipError_t launch_compact(const GridBufs &g, MatchBufs &m, PairState *ps, int32_t *scan_tmp, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipError_t e = exclusive_scan_i32(m.flag, m.kpos, g.ntot, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)m.flag, (const int32_t *)m.kpos, (const int32_t *)m.nn, m.kp, m.kq, m.ki, ps);
    return hipGetLastError();
}

}  // namespace lsr
