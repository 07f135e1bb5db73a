// Reciprocal test, quadruple consistency filter and compaction.
//
// Reciprocal: (i, nnQ(i)) is kept when nnP(nnQ(i)) = i.
// Consistency (Section IV, Algorithm 1: the four points of a hypothesis are
// picked at random from P and paired through the descriptor neighbours; the
// similar-polygon pre-rejection, used here as a filter): trial t fills slots
// s = 0..3 in order; slot s takes the first of up to 64 draws
// i = ((r >> 32) * N_P) >> 32 whose P point has a reciprocal correspondence
// and differs from the earlier slots, with r the n-th output of SplitMix64
// (Steele, Lea and Flood 2014) for the given seed and
// n = (t << 8) | (s << 6) | attempt; a slot with no such draw voids the
// trial.  The closed quadrilateral passes when every squared edge length
// ratio lies within tau^2 in both directions (FP64, a zero edge fails); the
// correspondences of a passing trial are flagged.
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

constexpr int TPB = 8192;    // trials per block (the trial table's granularity)
constexpr int CONS_THREADS[] = {256, 128, 512};   // block widths the autotuner picks from
constexpr int N_CONS_SHAPES = sizeof(CONS_THREADS) / sizeof(CONS_THREADS[0]);
constexpr int CH = 512;      // draw jobs (trial, slot) per result buffer; a wavefront owns two buffers
constexpr uint32_t VOID = 0xFFFFFFFFu;
constexpr int UNR = 4;       // draw attempts a lane makes per step (divides 64)
constexpr size_t LDS_CAP = 65536; // dynamic LDS a consistency block may take

// usable[g] = 1 for a P point with a reciprocal correspondence inside Q, or
// with any descriptor neighbour inside Q when mutual is NULL (scan input).
__global__ void __launch_bounds__(256) k_corr_usable(const Frag *frag, const Blk *blk, const int32_t *nn,
                                                     const uint8_t *mutual, int32_t *usable) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= P.n) return;
    bool u = false;
    if ((b.frag & 1) == 0 && P.partner >= 0 && (!mutual || mutual[P.off + i])) {
        int32_t j = nn[P.off + i];
        u = j >= 0 && j < frag[P.partner].n;
    }
    usable[P.off + i] = u ? 1 : 0;
}

// C packed in ascending P index at the scanned slots, one trial slot reading 32
// contiguous bytes: (p_i, q_nnQ(i)) and i; the pair's list start and length.
// Per 32 P points one word (bits of the points with a correspondence, packed
// position of the first of them): a draw's eligibility and its packed
// position are then one word read and a population count.
__global__ void __launch_bounds__(256) k_corr_pack(const Frag *frag, const Blk *blk, const int32_t *nn,
                                                   const int32_t *usable, const int32_t *cpos, float4 *cpack,
                                                   uint2 *cwords, PairState *ps) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    if ((b.frag & 1) || P.partner < 0) return;
    const Frag &Q = frag[P.partner];
    const int i = b.start + threadIdx.x;
    const int64_t gi = P.off + i;
    const bool u = i < P.n && usable[gi];
    const unsigned long long bal = __ballot(u);
    if (i < P.n && (i & 31) == 0) {
        const uint32_t bits = (uint32_t)(bal >> (threadIdx.x & 32));
        cwords[word_off(P, b.frag) + (i >> 5)] = make_uint2(bits, (uint32_t)cpos[gi]);
    }
    if (i >= P.n) return;
    if (i == P.n - 1) {
        ps[P.pair].c_off = cpos[P.off];
        ps[P.pair].c_cnt = cpos[gi] + usable[gi] - cpos[P.off];
    }
    if (!u) return;
    const int32_t j = nn[gi];
    const int64_t c = cpos[gi];
    cpack[2 * c] = make_float4(P.src[0][i], P.src[1][i], P.src[2][i], Q.src[0][j]);
    cpack[2 * c + 1] = make_float4(Q.src[1][j], Q.src[2][j], __int_as_float(i), 0.f);
}

// Correspondence words of a pair: for 32 consecutive P points the bits of
// those with a correspondence and the packed position of the first.  In LDS
// the two halves sit in separate arrays (a draw reads only the bits, with
// consecutive words in consecutive banks); in global memory as pairs.
struct LdsWords {
    const uint32_t *bits, *base;
    __device__ uint32_t b(uint32_t w) const { return bits[w]; }
    __device__ uint32_t p(uint32_t w) const { return base[w]; }
};
struct GlobalWords {
    const uint2 *w;
    __device__ uint32_t b(uint32_t k) const { return w[k].x; }
    __device__ uint32_t p(uint32_t k) const { return w[k].y; }
};

// Edge test of one drawn quadruple (positions in the packed C); flags the
// correspondences' P points when it passes.  The edges are tested in order
// and a correspondence is fetched only while every edge so far holds: the
// verdict is that of the full test, with fewer random gathers.
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

__device__ __forceinline__ uint64_t slot_state(uint64_t seed, int64_t t, int s) {
    return seed + ((((uint64_t)t << 8) | ((uint64_t)s << 6)) + 1ull) * GAMMA;
}

// Slot s of trial t drawn from its first attempt, skipping P points without
// a correspondence and the earlier slots' points x, y, w: the definition of
// a slot's draw.  The bulk draws below take the first eligible point and
// leave repeats (rare: about s in |C| per slot) to this.
template <class W>
__device__ uint32_t redraw(const W &words, uint32_t nP, uint64_t seed, int64_t t, int s, uint32_t x, uint32_t y,
                           uint32_t w) {
    uint64_t z = slot_state(seed, t, s);
    for (int a = 0; a < 64; ++a, z += GAMMA) {
        const uint32_t i = (uint32_t)(((uint64_t)splitmix64_hi(z) * nP) >> 32);
        if (((words.b(i >> 5) >> (i & 31)) & 1u) && i != x && i != y && i != w) return i;
    }
    return VOID;
}

// Trials whose four slot draws are complete: repeats redrawn in slot order,
// a void slot voids the trial, then the edge test.  r: the draws of trial
// u at r[4u .. 4u + 3]; lanes take trials lane, lane + 64, ...
template <class W>
__device__ int finish_trials(const W &words, uint32_t nP, uint64_t seed, int64_t t_first, int ntr,
                             const uint32_t *r, const float4 *cp, double t2, int32_t *fl) {
    int passed = 0;
    for (int u = threadIdx.x & 63; u < ntr; u += 64) {
        const uint4 d = *(const uint4 *)(r + 4 * u);
        uint32_t i0 = d.x, i1 = d.y, i2 = d.z, i3 = d.w;
        if (i0 == VOID || i1 == VOID || i2 == VOID || i3 == VOID) continue;
        const int64_t t = t_first + u;
        if (i1 == i0) i1 = redraw(words, nP, seed, t, 1, i0, i0, i0);
        if (i1 == VOID) continue;
        if (i2 == i0 || i2 == i1) i2 = redraw(words, nP, seed, t, 2, i0, i1, i1);
        if (i2 == VOID) continue;
        if (i3 == i0 || i3 == i1 || i3 == i2) i3 = redraw(words, nP, seed, t, 3, i0, i1, i2);
        if (i3 == VOID) continue;
        auto pos = [&](uint32_t i) {
            const uint32_t k = i >> 5;
            return (int)(words.p(k) + (uint32_t)__popc(words.b(k) & ((1u << (i & 31)) - 1u)));
        };
        passed += quad_test(cp, make_int4(pos(i0), pos(i1), pos(i2), pos(i3)), t2, fl);
    }
    return passed;
}

// One wavefront's trials [t0, t1), as 4 (t1 - t0) draw jobs (trial, slot) in
// trial-major order.  A lane holds one job (its SplitMix64 state and attempt
// count) and makes UNR attempts per step: the first attempt whose point has a
// correspondence ends the job (its point goes to the result buffer), as does
// the 64th (void).  A lane without a job claims the next in lane order
// (ballot + mbcnt), so lanes stay busy whatever their jobs' lengths.  Jobs
// fill two buffers of CH results; when every job of the older buffer has
// ended, the wavefront finishes its trials and the buffer is reused.  Job
// counters are per wavefront (fewer than 2^31 jobs: at most 4 TPB).
template <class W>
__device__ int wave_trials(const W &words, uint32_t nP, int64_t t0, int64_t t1, uint64_t seed, const float4 *cp,
                           uint32_t *res, double t2, int32_t *fl) {
    const int njobs = (int)(4 * (t1 - t0));
    int passed = 0;
    int next = 0;                  // next unclaimed job (wave-uniform)
    int oldest = 0;                // first job of the older buffer (wave-uniform, multiple of CH)
    int done_old = 0, done_new = 0;    // ended jobs in the older / newer buffer (wave-uniform)
    bool live = false;
    int j = 0, a = 0;
    uint64_t z = 0;
    for (;;) {
        const int limit = min(njobs, oldest + 2 * CH);
        const unsigned long long need = __ballot(!live);
        if (need && next < limit) {
            if (!live) {
                const int k = next + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                if (k < limit) {
                    live = true;
                    j = k;
                    a = 0;
                    z = slot_state(seed, t0 + (k >> 2), k & 3);
                }
            }
            next = min(limit, next + (int)__popcll(need));
        }
        bool fin = false;
        if (live) {
            // attempts a .. a + UNR - 1 (a multiple of UNR, 64 too): the first with a correspondence wins
            uint32_t pick = VOID;
#pragma unroll
            for (int u = UNR - 1; u >= 0; --u) {
                const uint32_t i = (uint32_t)(((uint64_t)splitmix64_hi(z + (uint64_t)u * GAMMA) * nP) >> 32);
                if ((words.b(i >> 5) >> (i & 31)) & 1u) pick = i;
            }
            if (pick != VOID || a == 64 - UNR) {
                res[j & (2 * CH - 1)] = pick;
                live = false;
                fin = true;
            } else {
                a += UNR;
                z += (uint64_t)UNR * GAMMA;
            }
        }
        const unsigned long long f_all = __ballot(fin);
        if (f_all) {
            const int n_old = __popcll(__ballot(fin && j < oldest + CH));
            done_old += n_old;
            done_new += __popcll(f_all) - n_old;
        }
        const int old_sz = min(CH, njobs - oldest);
        if (done_old == old_sz) {
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            passed += finish_trials(words, nP, seed, t0 + (oldest >> 2), old_sz >> 2, res + (oldest & (2 * CH - 1)),
                                    cp, t2, fl);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            oldest += CH;
            done_old = done_new;
            done_new = 0;
            if (oldest >= njobs) break;
        }
    }
    return passed;
}

// Block b takes trials [first, first + TPB) of its pair, split into
// contiguous ranges per wavefront.  Dynamic LDS: each wavefront's two result
// buffers, then room for lds_words correspondence words (bits, then
// positions); the pair's words go there when they fit, else the draws read
// them from global memory.  Fewer than four points with a correspondence: no
// trial can fill its four slots, none passes.
template <int CT>
__global__ void __launch_bounds__(CT) k_consistency(const Frag *frag, const TrialBlk *tb, const float4 *cpack,
                                                    const uint2 *cwords, int32_t *flag, double t2, uint64_t seed,
                                                    PairState *ps, int lds_words) {
    extern __shared__ uint4 dyn[];
    uint32_t *res = (uint32_t *)dyn + (threadIdx.x >> 6) * (2 * CH);
    uint32_t *sbits = (uint32_t *)dyn + (CT / 64) * (2 * CH);
    uint32_t *sbase = sbits + lds_words;
    const TrialBlk b = tb[blockIdx.x];
    const Frag &P = frag[2 * b.pair];
    const uint32_t nC = (uint32_t)ps[b.pair].c_cnt;
    const uint32_t nP = (uint32_t)P.n;
    if (nC < 4) return;
    const int64_t first = b.first, end = min(b.count, b.first + TPB);
    const int nw = (int)((nP + 31) >> 5);
    const uint2 *gw = cwords + word_off(P, 2 * b.pair);
    const bool in_lds = nw <= lds_words;
    if (in_lds) {
        for (int k = threadIdx.x; k < nw; k += CT) {
            const uint2 w = gw[k];
            sbits[k] = w.x;
            sbase[k] = w.y;
        }
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6;
    const int64_t per = (end - first + CT / 64 - 1) / (CT / 64);
    const int64_t t0 = first + wave * per, t1 = min(end, t0 + per);
    int passed = 0;
    if (t0 < t1) {
        int32_t *fl = flag + P.off;
        if (in_lds) passed = wave_trials(LdsWords{sbits, sbase}, nP, t0, t1, seed, cpack, res, t2, fl);
        else passed = wave_trials(GlobalWords{gw}, nP, t0, t1, seed, cpack, res, t2, fl);
    }
    // passing-trial count per pair (integer, order independent)
    for (int o = 32; o > 0; o >>= 1) passed += __shfl_xor(passed, o, 64);
    if ((threadIdx.x & 63) == 0 && passed) atomicAdd(&ps[b.pair].trials_passed, (unsigned long long)passed);
}

size_t corr_words(int64_t ntot, int nfrag) { return (size_t)(ntot >> 5) + (size_t)nfrag + 1; }

hipError_t launch_corr_pack(const GridBufs &g, MatchBufs &m, PairState *ps, bool one_way, int32_t *scan_tmp,
                            hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_corr_usable, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)m.nn, one_way ? nullptr : (const uint8_t *)m.mutual, m.flag);
    hipError_t e = exclusive_scan_i32(m.flag, m.kpos, g.ntot, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_corr_pack, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)m.nn, (const int32_t *)m.flag, (const int32_t *)m.kpos, m.cpack, m.cwords, ps);
    return hipGetLastError();
}

hipError_t launch_consistency(const GridBufs &g, MatchBufs &m, PairState *ps, const TrialBlk *tb, int ntb,
                              float tau, uint64_t seed, int shape, int32_t *scan_tmp, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipError_t e = launch_corr_pack(g, m, ps, false, scan_tmp, s);
    if (e != hipSuccess) return e;
    if ((e = fill<int32_t>(m.flag, 0, g.ntot, s)) != hipSuccess || ntb == 0) return e;
    double t2 = (double)tau * (double)tau;
    const Frag *fr = (const Frag *)g.frag;
    const float4 *cp = (const float4 *)m.cpack;
    const uint2 *cw = (const uint2 *)m.cwords;
    // words kept in LDS per block width: the pair's words when they fit beside the result buffers
    auto res_bytes = [](int ct) { return (size_t)(ct / 64) * 2 * CH * sizeof(uint32_t); };
    auto lw = [&](int ct) {
        return (int)std::min<int64_t>(((int64_t)g.max_np + 31) >> 5,
                                      (int64_t)((LDS_CAP - res_bytes(ct)) / (2 * sizeof(uint32_t))));
    };
    auto lds = [&](int ct) { return res_bytes(ct) + (size_t)lw(ct) * 2 * sizeof(uint32_t); };
    switch (shape) {
    case 0: hipLaunchKernelGGL(k_consistency<CONS_THREADS[0]>, dim3(ntb), dim3(CONS_THREADS[0]), lds(CONS_THREADS[0]),
                               s, fr, tb, cp, cw, m.flag, t2, seed, ps, lw(CONS_THREADS[0])); break;
    case 1: hipLaunchKernelGGL(k_consistency<CONS_THREADS[1]>, dim3(ntb), dim3(CONS_THREADS[1]), lds(CONS_THREADS[1]),
                               s, fr, tb, cp, cw, m.flag, t2, seed, ps, lw(CONS_THREADS[1])); break;
    case 2: hipLaunchKernelGGL(k_consistency<CONS_THREADS[2]>, dim3(ntb), dim3(CONS_THREADS[2]), lds(CONS_THREADS[2]),
                               s, fr, tb, cp, cw, m.flag, t2, seed, ps, lw(CONS_THREADS[2])); break;
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
