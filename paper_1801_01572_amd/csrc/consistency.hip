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
constexpr int RING = 128;    // drawn quadruples parked per wavefront before their edge tests
constexpr int LDS_WORDS = 6144;   // correspondence words a block keeps in LDS (P fragments <= 196,608 points)

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

// One wavefront's trials [t, t_end).  Every lane runs draws without waiting
// for the others: a lane holds one trial (slot s, attempt state z, the P
// indices and packed positions accepted so far) and takes one draw per step;
// a lane whose trial completes or is void takes the wavefront's next trial
// (ballot + mbcnt).  Complete quadruples are parked in the wavefront's LDS
// ring and edge-tested 64 at a time, so that the gathers of the test run
// with every lane busy.  Words: the pair's correspondence words (LDS or
// global memory).
template <class WordPtr>
__device__ int wave_trials(WordPtr words, uint32_t nP, int64_t t, int64_t t_end, uint64_t seed, const float4 *cp,
                           int4 *ring, double t2, int32_t *fl) {
    const int lane = threadIdx.x & 63;
    int passed = 0;
    int head = 0, cnt = 0;                       // ring (wave-uniform)
    int64_t next = t;                            // wave's next unclaimed trial (wave-uniform)
    bool live = false;
    int s = 0, a = 0;
    uint32_t id0 = 0, id1 = 0, id2 = 0;
    int4 pos = make_int4(0, 0, 0, 0);
    uint64_t zs = 0, z = 0;
    for (;;) {
        // lanes without a trial claim the next ones in lane order
        const unsigned long long need = __ballot(!live);
        if (need && next < t_end) {
            if (!live) {
                const int64_t k = next + (int64_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                if (k < t_end) {
                    live = true;
                    s = 0;
                    a = 0;
                    zs = seed + (((uint64_t)k << 8) + 1ull) * GAMMA;
                    z = zs;
                }
            }
            next += __popcll(need);
        }
        bool done = false;
        if (live) {
            const uint32_t i = (uint32_t)(((uint64_t)splitmix64_hi(z) * nP) >> 32);
            const uint2 w = words[i >> 5];
            const uint32_t below = w.x & ((1u << (i & 31)) - 1u);
            const bool ok = ((w.x >> (i & 31)) & 1u) && !(s > 0 && i == id0) && !(s > 1 && i == id1) &&
                            !(s > 2 && i == id2);
            if (ok) {
                const int p = (int)(w.y + (uint32_t)__popc(below));
                if (s == 0) { id0 = i; pos.x = p; }
                else if (s == 1) { id1 = i; pos.y = p; }
                else if (s == 2) { id2 = i; pos.z = p; }
                else { pos.w = p; done = true; }
                ++s;
                a = 0;
                zs += 64ull * GAMMA;
                z = zs;
            } else if (++a == 64) {
                live = false;                    // void trial
            } else {
                z += GAMMA;
            }
            if (done) live = false;
        }
        // park complete quadruples
        const unsigned long long put = __ballot(done);
        if (done) {
            const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(put >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)put, 0u));
            ring[(head + cnt + r) & (RING - 1)] = pos;
        }
        cnt += __popcll(put);
        const bool any_live = __ballot(live) != 0ull;
        const bool more = any_live || next < t_end;
        if (cnt >= 64 || (!more && cnt > 0)) {
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int take = cnt < 64 ? cnt : 64;
            if (lane < take) passed += quad_test(cp, ring[(head + lane) & (RING - 1)], t2, fl);
            head = (head + take) & (RING - 1);
            cnt -= take;
            __builtin_amdgcn_wave_barrier();
        }
        if (!more && cnt == 0) break;
    }
    return passed;
}

// Block b takes trials [first, first + TPB) of its pair, split into
// contiguous ranges per wavefront.  Dynamic LDS: the wavefronts' rings, then
// room for lds_words correspondence words; the pair's words go there when
// they fit, else the draws read them from global memory.  Fewer than four
// points with a correspondence: no trial can fill its four slots, none
// passes.
template <int CT>
__global__ void __launch_bounds__(CT) k_consistency(const Frag *frag, const TrialBlk *tb, const float4 *cpack,
                                                    const uint2 *cwords, int32_t *flag, double t2, uint64_t seed,
                                                    PairState *ps, int lds_words) {
    extern __shared__ int4 dyn[];
    int4 *ring = dyn + (threadIdx.x >> 6) * RING;
    uint2 *sw = (uint2 *)(dyn + (CT / 64) * RING);
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
        for (int k = threadIdx.x; k < nw; k += CT) sw[k] = gw[k];
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6;
    const int64_t per = (end - first + CT / 64 - 1) / (CT / 64);
    const int64_t t0 = first + wave * per, t1 = min(end, t0 + per);
    int passed = 0;
    if (t0 < t1) {
        int32_t *fl = flag + P.off;
        if (in_lds) passed = wave_trials<const uint2 *>(sw, nP, t0, t1, seed, cpack, ring, t2, fl);
        else passed = wave_trials<const uint2 *>(gw, nP, t0, t1, seed, cpack, ring, t2, fl);
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
    const int lw = (int)std::min<int64_t>(((int64_t)g.max_np + 31) >> 5, LDS_WORDS);
    auto lds = [&](int ct) { return (size_t)(ct / 64) * RING * sizeof(int4) + (size_t)lw * sizeof(uint2); };
    switch (shape) {
    case 0: hipLaunchKernelGGL(k_consistency<CONS_THREADS[0]>, dim3(ntb), dim3(CONS_THREADS[0]), lds(CONS_THREADS[0]),
                               s, fr, tb, cp, cw, m.flag, t2, seed, ps, lw); break;
    case 1: hipLaunchKernelGGL(k_consistency<CONS_THREADS[1]>, dim3(ntb), dim3(CONS_THREADS[1]), lds(CONS_THREADS[1]),
                               s, fr, tb, cp, cw, m.flag, t2, seed, ps, lw); break;
    case 2: hipLaunchKernelGGL(k_consistency<CONS_THREADS[2]>, dim3(ntb), dim3(CONS_THREADS[2]), lds(CONS_THREADS[2]),
                               s, fr, tb, cp, cw, m.flag, t2, seed, ps, lw); break;
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
