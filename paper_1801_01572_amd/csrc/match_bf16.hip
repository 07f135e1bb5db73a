// Descriptor nearest neighbours screened on the matrix cores (bf16 inputs,
// float32 accumulation), re-ranked exactly, with a proof that the re-ranked
// winner is the float32 scan's winner, or else a float32 rescan of the row.
//
// Packing.  Each 11-bin block of an FPFH descriptor sums to 1, so a distance
// between two descriptors only sees the sum-free part of each block: with the
// Helmert contrasts h_k = (x_0 + .. + x_{k-1} - k x_k) / sqrt(k (k+1)),
// k = 1..10, the 33-vector maps to y (30 numbers) with |F_i - F_j| = |y_i - y_j|.
// y is centred on the pair's mean descriptor (distances unchanged, smaller
// magnitudes).  y is split into bf16 hi + lo parts (hi + lo within 2^-18 of
// y).  A candidate row is [y_hi, c_hi, c_lo | y_lo, 0, 0] with
// c_hi + c_lo = -|y_j|^2 / 2; a query enters rounded once, as [y_hi, 1, 1].
// Two chained 16x16x32 bf16 MFMAs (hi_cand.hi_query, lo_cand.hi_query) give
//   t_ij = yh_i . y_j - |y_j|^2 / 2,   yh_i = bf16(y_i),
// while the exact score is s_ij = y_i . y_j - |y_j|^2 / 2 = (|y_i|^2 - D_ij) / 2.
// With d_i = y_i - yh_i, s_ij - t_ij = d_i . y_j = c_i + d_i . (y_j - y_i),
// c_i = d_i . y_i: a per-query constant (no effect on the ranking) plus a
// term bounded by |d_i| sqrt(D_ij), small exactly for the candidates that
// compete for the minimum.
//
// Screen.  A wave owns 4 blocks of 16 queries and sweeps the partner's rows
// 16 at a time from LDS (chunks of 128 rows, double buffered).  Lane l sees
// query column l % 16 and candidate rows 4 (l / 16) + {0..3} of every tile
// (lane group g = l / 16).  Per tile a lane takes the maximum of its four
// scores; across tiles it keeps the best tile and the second-best tile maximum.
//
// Certification.  The 16 rows of the four groups' best tiles are re-ranked
// with the exact float32 distance d2_row, giving D*.  A row j outside them has
// a screened score t_ij <= A2, the largest second-best tile maximum.  Only
// rows with D_ij <= D* + slack can matter; those have
// |y_j| <= |y_i| + sqrt(D* + slack) = R and s_ij <= t_ij + c_i + E with
// E = |d_i| sqrt(D* + slack) + 2^-15 (|y_i| R + R^2 / 2) (the second term
// covers the candidate split, the norm slots and float32 accumulation, with
// margin).  If D* + slack < |y_i|^2 - 2 (A2 + c_i + E) no outside row can win
// and D* with its index is the float32 scan's answer.  Otherwise the row goes
// to a second screen that collects every candidate whose screened score
// reaches theta = (|y_i|^2 - D* - slack) / 2 - c_i - E (a superset of all rows
// that can tie or beat D*), and those are re-ranked exactly.  Only a row with
// more than LCAP such candidates is rescanned in float32.
#include <rocprim/device/device_radix_sort.hpp>

#include "match_common.h"

namespace lsr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Screen shapes: tile edge T (16: 16x16x32 MFMAs, 32: 32x32x16 MFMAs), SW
// waves per block x SQB T-query blocks per wave = 256 queries per block (one
// block per 256 rows of a fragment, any variant); CH T-row tiles per LDS
// chunk; prune: skip the partner's chunks that provably cannot matter (the
// pruned screen below).  The variant is chosen by the autotuner.
struct ScreenShape { int t, sw, sqb, ch, prune; };
constexpr ScreenShape SCREEN_SHAPES[] = {{16, 4, 4, 8, 0}, {16, 4, 4, 4, 0}, {16, 8, 2, 8, 0}, {16, 8, 2, 4, 0},
                                         {32, 4, 2, 4, 0}, {16, 4, 4, 8, 1}, {16, 2, 8, 8, 0}, {16, 2, 8, 4, 0}};
constexpr int N_SCREEN_SHAPES = sizeof(SCREEN_SHAPES) / sizeof(SCREEN_SHAPES[0]);
constexpr int PAD_ROWS = 128;      // fragments' packed rows are padded to a multiple of this
constexpr int LCAP = 32;           // candidates collected per uncertified row

__device__ __forceinline__ uint16_t f2bf(float f) {     // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint32_t lanes_below_w(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

struct ScreenScratch {
    float *mean;          // (nfrag/2 + 1) x 32: projected centring vector per pair
    float4 *yq;           // pk_rows: (|y|^2, c = d . y, |d|, 0) with d = y - bf16(y)
    int32_t *c1;          // ntot x 4: best tile per lane group
    float *v2;            // ntot x 4: second-best tile maximum per lane group
    float *v1;            // ntot x 4: best tile maximum per lane group
    int32_t *fb_row;      // ntot: uncertified rows, per fragment from Frag::off
    float *thr;           // ntot: collection threshold of each uncertified row
    int32_t *fb_cnt;      // nfrag
    int32_t *lst;         // list slots x LCAP
    int32_t *lst_cnt;     // list slots
    int32_t *full_row, *full_frag, *full_cnt;
    int32_t *lmark, *lpos;// ntot: uncertified rows marked at their packed rows, and the marks' exclusive scan
    int32_t *fb_row2;     // ntot: the uncertified rows of each fragment in packed-row order
    float *thr2;          // ntot: their thresholds
    int32_t *stmp;        // scan scratch
    // descriptor-space row order (see "Row order" below)
    float *pca;           // (nfrag/2 + 1) x 96: three principal directions (30 each) and their key scales
    uint64_t *key0, *key1;// ntot: (fragment, Hilbert key) sort keys
    uint32_t *idx0;       // ntot: point index (sort values in)
    int32_t *perm;        // ntot: packed row r of a fragment holds its point perm[off + r] (sort values out)
    int32_t *rinv;        // ntot: packed row of each point
    void *sort_tmp;
    size_t sort_bytes;
    uint16_t *cpk;        // centroid rows of the partner chunks (pruned screen), packed like candidate rows
    float4 *cst;          // per centroid row: (radius, score offset bound, max |y|^2 + max h, |centroid|^2)
};

// list slots of fragment f: [off/4 + 64 f, ... + n/4 + 64)
__device__ __forceinline__ int64_t lst_base(const Frag &F, int f) { return F.off / 4 + 64 * (int64_t)f; }
__device__ __forceinline__ int32_t lst_cap(const Frag &F) { return F.n / 4 + 64; }
static int64_t lst_slots(const GridBufs &g) { return g.ntot / 4 + 64 * (int64_t)g.nfrag + 64; }
// centroid rows of fragment f: [pk_off / 128 + 128 f, + ceil(chunks / 128) 128), chunks = padded rows / 128
__device__ __forceinline__ int64_t cent_base(const Frag &F, int f) { return F.pk_off / PAD_ROWS + 128 * (int64_t)f; }
// sort keys: fragment index above a 25-bit Hilbert key (2^24 marks an invalid descriptor)
static int sort_end_bit(int nfrag) {
    int b = 1;
    while ((1 << b) < nfrag + 1 && b < 31) ++b;
    return 25 + b;
}
static int64_t cent_rows(const GridBufs &g) { return g.pk_rows / PAD_ROWS + 128 * (int64_t)g.nfrag + 128; }

static ScreenScratch carve(void *base, const GridBufs &g, size_t *bytes) {
    char *p = (char *)base;
    size_t tot = 0;
    auto take = [&](size_t n) { char *r = p; size_t a = (n + 255) & ~size_t(255); p += a; tot += a; return r; };
    const size_t n1 = (size_t)std::max<int64_t>(g.ntot, 1);
    ScreenScratch s;
    s.mean = (float *)take(sizeof(float) * 32 * (size_t)(g.nfrag / 2 + 1));
    s.yq = (float4 *)take(sizeof(float4) * (size_t)std::max<int64_t>(g.pk_rows, 1));
    s.c1 = (int32_t *)take(sizeof(int32_t) * 4 * n1);
    s.v2 = (float *)take(sizeof(float) * 4 * n1);
    s.v1 = (float *)take(sizeof(float) * 4 * n1);
    s.fb_row = (int32_t *)take(sizeof(int32_t) * n1);
    s.thr = (float *)take(sizeof(float) * n1);
    s.fb_cnt = (int32_t *)take(sizeof(int32_t) * (size_t)std::max(g.nfrag, 1));
    s.lst = (int32_t *)take(sizeof(int32_t) * LCAP * (size_t)lst_slots(g));
    s.lst_cnt = (int32_t *)take(sizeof(int32_t) * (size_t)lst_slots(g));
    s.full_row = (int32_t *)take(sizeof(int32_t) * n1);
    s.full_frag = (int32_t *)take(sizeof(int32_t) * n1);
    s.full_cnt = (int32_t *)take(256);
    s.lmark = (int32_t *)take(sizeof(int32_t) * n1);
    s.lpos = (int32_t *)take(sizeof(int32_t) * n1);
    s.fb_row2 = (int32_t *)take(sizeof(int32_t) * n1);
    s.thr2 = (float *)take(sizeof(float) * n1);
    s.stmp = (int32_t *)take(sizeof(int32_t) * scan_tmp_elems((int64_t)n1));
    s.pca = (float *)take(sizeof(float) * 96 * (size_t)(g.nfrag / 2 + 1));
    s.key0 = (uint64_t *)take(sizeof(uint64_t) * n1);
    s.key1 = (uint64_t *)take(sizeof(uint64_t) * n1);
    s.idx0 = (uint32_t *)take(sizeof(uint32_t) * n1);
    s.perm = (int32_t *)take(sizeof(int32_t) * n1);
    s.rinv = (int32_t *)take(sizeof(int32_t) * n1);
    s.sort_bytes = 0;
    (void)rocprim::radix_sort_pairs(nullptr, s.sort_bytes, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                    (uint32_t *)nullptr, (uint32_t *)nullptr, n1, 0, sort_end_bit(g.nfrag));
    s.sort_tmp = take(s.sort_bytes);
    const size_t ncent = (size_t)cent_rows(g);
    s.cpk = (uint16_t *)take(sizeof(uint16_t) * PK * ncent);
    s.cst = (float4 *)take(sizeof(float4) * ncent);
    if (bytes) *bytes = tot;
    return s;
}

size_t match_bf16_scratch(const GridBufs &g, int64_t pk_rows) {
    GridBufs h = g;
    h.pk_rows = pk_rows;
    size_t bytes = 0;
    (void)carve(nullptr, h, &bytes);
    return bytes;
}

// ---------------------------------------------------------------- centring

// Helmert contrasts of one 11-bin block (orthonormal, orthogonal to all-ones).
__device__ __forceinline__ void helmert11(const float *x, float *h) {
    float s = x[0];
#pragma unroll
    for (int k = 1; k < NB; ++k) {
        h[k - 1] = (s - (float)k * x[k]) * rsqrtf((float)(k * (k + 1)));
        s += x[k];
    }
}

// One block per pair: the mean of up to 4096 valid descriptors of each
// fragment (any centre gives the same distances; a nearby one keeps the
// screen's magnitudes small), projected.  Fixed summation order.
__global__ void __launch_bounds__(256) k_desc_mean(const Frag *frag, int nfrag, const float *F, const int32_t *valid,
                                                   float *mean_out) {
    __shared__ float sh[4][34];
    const int b = blockIdx.x;
    float acc[34];
#pragma unroll
    for (int c = 0; c < 34; ++c) acc[c] = 0.f;
    for (int f = 2 * b; f <= 2 * b + 1 && f < nfrag; ++f) {
        const Frag &Fr = frag[f];
        int lim = min(Fr.n, 4096);
        for (int i = threadIdx.x; i < lim; i += 256) {
            if (!valid[Fr.off + i]) continue;
            const float *x = F + (Fr.off + i) * FD;
#pragma unroll
            for (int c = 0; c < FD; ++c) acc[c] += x[c];
            acc[33] += 1.f;
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 34; ++c) {
        float v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[w][c] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m[34];
        for (int c = 0; c < 34; ++c) m[c] = ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c];
        float inv = m[33] > 0 ? 1.0f / m[33] : 0.f;
        for (int c = 0; c < FD; ++c) m[c] *= inv;
        float h[30];
        for (int k = 0; k < 3; ++k) helmert11(m + NB * k, h + 10 * k);
        for (int c = 0; c < 30; ++c) mean_out[32 * b + c] = h[c];
        mean_out[32 * b + 30] = 0.f;         // largest projection error of the pair's P rows (k_pack)
        mean_out[32 * b + 31] = 0.f;         // ... and of its Q rows
    }
}

// Point i of a fragment goes to packed row rinv[off + i]; thread t < n takes
// point t (rows read in order, whole 128-byte rows written), a thread in
// [n, padded n) writes padding row t.  yq stays indexed by point.  The bf16
// halves are packed two to a word as they are made, and the pair's largest
// projection error takes one atomic per wavefront.
__global__ void __launch_bounds__(256) k_pack(const Frag *frag, const Blk *blk, const float *F, const int32_t *valid,
                                              float *mean, const int32_t *rinv, uint16_t *pk, float4 *yq) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fr = frag[b.frag];
    const int t = b.start + threadIdx.x;
    const int npad = (Fr.n + PAD_ROWS - 1) / PAD_ROWS * PAD_ROWS;
    const bool active = t < npad;
    const int i = t;
    uint32_t hw[16], lw[16];                                  // bf16 pairs: hi slots 0-31, lo slots 0-31
    float n2 = 0.f, dd = 0.f, delta = 0.f;
    double dy = 0.0;
    const bool v = t < Fr.n && valid[Fr.off + i];
    if (v) {
        const float *x = F + (Fr.off + i) * FD;
        const float *m = mean + 32 * (b.frag >> 1);
        float h[30];
        float xb[FD];
#pragma unroll
        for (int c = 0; c < FD; ++c) xb[c] = x[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) helmert11(xb + NB * k, h + 10 * k);
#pragma unroll
        for (int c = 0; c < 30; ++c) {
            h[c] -= m[c];
            n2 = fmaf(h[c], h[c], n2);
            const uint16_t hc = f2bf(h[c]);
            const float d = h[c] - bf2f(hc);                 // exact
            const uint16_t lc = f2bf(d);
            dd = fmaf(d, d, dd);
            dy += (double)d * (double)h[c];
            if (c & 1) { hw[c >> 1] |= (uint32_t)hc << 16; lw[c >> 1] |= (uint32_t)lc << 16; }
            else { hw[c >> 1] = hc; lw[c >> 1] = lc; }
        }
        const float cc = -0.5f * n2;
        const uint16_t c0 = f2bf(cc);
        hw[15] = c0 | ((uint32_t)f2bf(cc - bf2f(c0)) << 16);
        // projection error: |y - y*| with y* the FP64 Helmert projection of the same float
        // descriptor minus the same centre (rounded up); the certificate widens by it
        double e2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double sd = xb[NB * k];
#pragma unroll
            for (int q = 1; q < NB; ++q) {
                const double hd = (sd - (double)q * (double)xb[NB * k + q]) / sqrt((double)(q * (q + 1)));
                const double ed = (double)h[10 * k + q - 1] - (hd - (double)m[10 * k + q - 1]);
                e2 += ed * ed;
                sd += (double)xb[NB * k + q];
            }
        }
        delta = (float)(sqrt(e2) * (1.0 + 1e-6)) + 1e-15f;
    } else {
#pragma unroll
        for (int w = 0; w < 15; ++w) { hw[w] = 0; lw[w] = 0; }
        hw[15] = f2bf(-1.0e30f);
    }
    lw[15] = 0;
    // the pair's largest projection error (non-negative floats order as their bits)
    float dm = delta;
    for (int o = 32; o > 0; o >>= 1) dm = fmaxf(dm, __shfl_xor(dm, o, 64));
    if ((threadIdx.x & 63) == 0 && dm > 0.f)
        atomicMax((unsigned int *)(mean + 32 * (b.frag >> 1) + 30 + (b.frag & 1)), __float_as_uint(dm));
    if (!active) return;
    const int r = t < Fr.n ? rinv[Fr.off + t] : t;
    uint4 *dst = (uint4 *)(pk + (Fr.pk_off + r) * PK);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = make_uint4(hw[4 * q], hw[4 * q + 1], hw[4 * q + 2], hw[4 * q + 3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[4 + q] = make_uint4(lw[4 * q], lw[4 * q + 1], lw[4 * q + 2], lw[4 * q + 3]);
    if (t < Fr.n) yq[Fr.pk_off + i] = make_float4(n2, (float)dy, sqrtf(dd) * 1.0001f, delta);
}

// ---------------------------------------------------------------- row order
//
// Row order.  Each fragment's packed rows are sorted by a Hilbert key of their
// first three principal components (8 bits each, over the pair's descriptor
// sample), so that a 256-row query block and a 128-row candidate chunk are
// each compact in descriptor space.  The order changes no result: every
// kernel maps packed rows back to points, and ties are broken by point index.
// The pruned screen then bounds a whole chunk at once through its centroid.

// One block per pair: the covariance of the centred, projected descriptors
// of the same sample as the centring (up to 4096 valid rows per fragment),
// then its three leading eigenvectors by power iteration with deflation.
// Key scale of component c: 128 / (3 sigma_c), so +-3 sigma spans the 8 bits.
__global__ void __launch_bounds__(256) k_pca(const Frag *frag, int nfrag, const float *F, const int32_t *valid,
                                             const float *mean, float *pca) {
    __shared__ float sy[64][31];
    __shared__ float cv[30][31];
    __shared__ int cnt_sh;
    const int b = blockIdx.x, tid = threadIdx.x;
    const float *m = mean + 32 * b;
    // entries e = tid, tid + 256 of the upper triangle (465 entries)
    int ea[2], ec[2];
    for (int u = 0; u < 2; ++u) {
        int e = tid + 256 * u, a = 0;
        while (e >= 30 - a && a < 30) { e -= 30 - a; ++a; }
        ea[u] = a < 30 ? a : -1;
        ec[u] = a + e;
    }
    float acc[2] = {0.f, 0.f};
    int cnt = 0;
    for (int f = 2 * b; f <= 2 * b + 1 && f < nfrag; ++f) {
        const Frag &Fr = frag[f];
        const int lim = min(Fr.n, 4096);
        for (int i0 = 0; i0 < lim; i0 += 64) {
            if (tid < 64) {
                const int i = i0 + tid;
                float h[30];
                const bool v = i < lim && valid[Fr.off + i];
                if (v) {
                    const float *x = F + (Fr.off + i) * FD;
                    float xb[FD];
                    for (int c = 0; c < FD; ++c) xb[c] = x[c];
                    for (int k = 0; k < 3; ++k) helmert11(xb + NB * k, h + 10 * k);
                }
                for (int c = 0; c < 30; ++c) sy[tid][c] = v ? h[c] - m[c] : 0.f;
                cnt += v ? 1 : 0;
            }
            __syncthreads();
            for (int u = 0; u < 2; ++u)
                if (ea[u] >= 0)
                    for (int r = 0; r < 64; ++r) acc[u] = fmaf(sy[r][ea[u]], sy[r][ec[u]], acc[u]);
            __syncthreads();
        }
    }
    for (int u = 0; u < 2; ++u)
        if (ea[u] >= 0) { cv[ea[u]][ec[u]] = acc[u]; cv[ec[u]][ea[u]] = acc[u]; }
    if (tid < 64) {
        int c = cnt;
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (tid == 0) cnt_sh = c;
    }
    __syncthreads();
    if (tid >= 64) return;
    const int lane = tid;
    const float n = (float)max(cnt_sh, 1);
    float *out = pca + 96 * b;
    for (int comp = 0; comp < 3; ++comp) {
        float v = lane < 30 ? 1.0f + 0.01f * (float)lane * (float)(comp + 1) : 0.f;
        float lam = 0.f;
        for (int it = 0; it < 64; ++it) {
            float w = 0.f;
            for (int k = 0; k < 30; ++k) {
                const float vk = __shfl(v, k, 64);
                if (lane < 30) w = fmaf(cv[lane][k], vk, w);
            }
            float n2 = w * w;
            for (int o = 32; o > 0; o >>= 1) n2 += __shfl_xor(n2, o, 64);
            if (!(n2 > 0.f)) break;
            lam = sqrtf(n2);
            const float vn = w / lam;
            // stop once the direction moves by less than 1e-4 (the keys only
            // order rows; any direction is correct)
            float dv = (vn - v) * (vn - v);
            for (int o = 32; o > 0; o >>= 1) dv += __shfl_xor(dv, o, 64);
            v = vn;
            if (dv < 1e-8f) break;
        }
        // deflate: cv -= lam v v^T
        for (int k = 0; k < 30; ++k) {
            const float vk = __shfl(v, k, 64);
            if (lane < 30) cv[lane][k] -= lam * v * vk;
        }
        if (lane < 30) out[30 * comp + lane] = v;
        if (lane == 0) out[90 + comp] = lam > 0.f ? 128.0f / (3.0f * sqrtf(lam / n)) : 0.f;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__device__ __forceinline__ uint32_t spread3(uint32_t x) {      // bit k of x to bit 3k (8 bits)
    x &= 0xFFu;
    x = (x | (x << 8)) & 0x00F00Fu;
    x = (x | (x << 4)) & 0x0C30C3u;
    x = (x | (x << 2)) & 0x249249u;
    return x;
}

// Sort key of each point: fragment index above the 24-bit Hilbert index of its
// three quantised projections (2^24 for an invalid descriptor, so those rows go
// last).  The Hilbert curve never jumps, so a run of 128 consecutive keys is a
// more compact chunk than a Morton run (48.0 -> 46.9% of the chunk visits).
__global__ void __launch_bounds__(256) k_mkey(const Frag *frag, const Blk *blk, const float *F, const int32_t *valid,
                                              const float *mean, const float *pca, uint64_t *key, uint32_t *idx) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fr = frag[b.frag];
    const int i = b.start + threadIdx.x;
    if (i >= Fr.n) return;
    uint32_t mk = 1u << 24;
    if (valid[Fr.off + i]) {
        const float *x = F + (Fr.off + i) * FD;
        const float *m = mean + 32 * (b.frag >> 1);
        const float *pc = pca + 96 * (b.frag >> 1);
        float xb[FD], h[30];
#pragma unroll
        for (int c = 0; c < FD; ++c) xb[c] = x[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) helmert11(xb + NB * k, h + 10 * k);
        float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 30; ++c) {
            const float y = h[c] - m[c];
#pragma unroll
            for (int k = 0; k < 3; ++k) p[k] = fmaf(y, pc[30 * k + c], p[k]);
        }
        uint32_t q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float t = floorf(fmaf(p[k], pc[90 + k], 128.0f));
            t = fminf(fmaxf(t, 0.0f), 255.0f);           // NaN -> 0 through fmax
            q[k] = (uint32_t)t;
        }
        {   // Hilbert order: the coordinates in transposed form (Skilling 2004), then interleaved
            for (uint32_t Q = 128u; Q > 1u; Q >>= 1) {
                const uint32_t P = Q - 1u;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (q[k] & Q) {
                        q[0] ^= P;
                    } else {
                        const uint32_t t = (q[0] ^ q[k]) & P;
                        q[0] ^= t;
                        q[k] ^= t;
                    }
                }
            }
            q[1] ^= q[0];
            q[2] ^= q[1];
            uint32_t t = 0u;
            for (uint32_t Q = 128u; Q > 1u; Q >>= 1)
                if (q[2] & Q) t ^= Q - 1u;
            q[0] ^= t; q[1] ^= t; q[2] ^= t;
        }
        mk = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    }
    key[Fr.off + i] = ((uint64_t)b.frag << 25) | mk;
    idx[Fr.off + i] = (uint32_t)i;
}

// rinv[off + perm[off + r]] = r
__global__ void __launch_bounds__(256) k_rinv(const Frag *frag, const Blk *blk, const int32_t *perm, int32_t *rinv) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fr = frag[b.frag];
    const int r = b.start + threadIdx.x;
    if (r >= Fr.n) return;
    rinv[Fr.off + perm[Fr.off + r]] = r;
}

// One wavefront per 128-row chunk of packed rows: the centroid mu of the valid
// rows y~ = hi + lo (float32, exact), split like a candidate row, and the
// chunk's bounds for the pruned screen: radius rho >= |y~_j - mu~|, score
// offset delta >= |y~_j|^2 / 2 - h_j (h_j = -(c_hi + c_lo), FP64, rounded up),
// max |y~_j|^2 + max h_j, and |mu~|^2.  A chunk without valid rows gets
// radius -1 and a centroid that no query can approach.  The last chunk's
// wavefront also writes the padding centroid rows.
__global__ void __launch_bounds__(128) k_chunk_stats(const Frag *frag, const Blk *blk, const uint16_t *pk,
                                                     uint16_t *cpk, float4 *cst) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fr = frag[b.frag];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nch = (Fr.n + PAD_ROWS - 1) / PAD_ROWS;
    const int k = b.start / PAD_ROWS + wv;                 // 256-point block, two wavefronts: chunks start/128 + {0, 1}
    if (k >= nch) return;
    const int64_t cb = cent_base(Fr, b.frag);
    // one row (lane + 64 u of the chunk): y~ = hi + lo, h = -(c_hi + c_lo), valid
    auto load = [&](int u, float *y, float &h) {
        const uint4 *row4 = (const uint4 *)(pk + (Fr.pk_off + (int64_t)k * PAD_ROWS + lane + 64 * u) * PK);
        uint4 w4[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) w4[q] = row4[q];
        const uint16_t *row = (const uint16_t *)w4;
        const float chi = bf2f(row[30]), clo = bf2f(row[31]);
        h = -(chi + clo);
#pragma unroll
        for (int c = 0; c < 30; ++c) y[c] = bf2f(row[c]) + bf2f(row[32 + c]);
        return chi > -1.0e29f;
    };
    // the lane's two rows, loaded once for both passes
    float yr[2][30], hr[2];
    bool vr[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) vr[u] = load(u, yr[u], hr[u]);
    float s[30];
#pragma unroll
    for (int c = 0; c < 30; ++c) s[c] = 0.f;
    int nv = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (!vr[u]) continue;
#pragma unroll
        for (int c = 0; c < 30; ++c) s[c] += yr[u][c];
        ++nv;
    }
    for (int o = 32; o > 0; o >>= 1) nv += __shfl_xor(nv, o, 64);
    uint16_t mh[32], ml[32];
    float mu[30], mu2 = 0.f;
#pragma unroll
    for (int c = 0; c < 30; ++c) {
        float t = s[c];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        t = nv > 0 ? t / (float)nv : 0.f;
        mh[c] = f2bf(t);
        ml[c] = f2bf(t - bf2f(mh[c]));
        mu[c] = bf2f(mh[c]) + bf2f(ml[c]);
        mu2 = fmaf(mu[c], mu[c], mu2);
    }
    float rho = 0.f, ym = 0.f, hm = 0.f;
    double del = -1.0e300;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (!vr[u]) continue;
        const float *y = yr[u];
        const float h = hr[u];
        float d2 = 0.f, n2f = 0.f;
        double n2 = 0.0;
#pragma unroll
        for (int c = 0; c < 30; ++c) {
            const float d = y[c] - mu[c];
            d2 = fmaf(d, d, d2);
            n2f = fmaf(y[c], y[c], n2f);
            n2 = fma((double)y[c], (double)y[c], n2);
        }
        rho = fmaxf(rho, sqrtf(d2));
        ym = fmaxf(ym, n2f);
        hm = fmaxf(hm, h);
        del = fmax(del, 0.5 * n2 - (double)h);
    }
    for (int o = 32; o > 0; o >>= 1) {
        rho = fmaxf(rho, __shfl_xor(rho, o, 64));
        ym = fmaxf(ym, __shfl_xor(ym, o, 64));
        hm = fmaxf(hm, __shfl_xor(hm, o, 64));
        del = fmax(del, __shfl_xor(del, o, 64));
    }
    const float cc = -0.5f * mu2;
    if (lane == 0) {
        float4 st;
        if (nv > 0) {
            float df = (float)del;
            df += fabsf(df) * 2.4e-7f + 1.0e-30f;                // rounded up
            st = make_float4(rho * (1.0f + 1.0e-6f) + 1.0e-30f, df, (ym + hm) * (1.0f + 1.0e-6f),
                             mu2 * (1.0f + 1.0e-6f));
        } else {
            st = make_float4(-1.0f, 0.f, 0.f, 0.f);
        }
        cst[cb + k] = st;
        uint16_t *dst = cpk + (cb + k) * PK;
        for (int c = 0; c < 30; ++c) { dst[c] = mh[c]; dst[32 + c] = ml[c]; }
        const uint16_t chi = nv > 0 ? f2bf(cc) : f2bf(-1.0e30f);
        dst[30] = chi;
        dst[31] = nv > 0 ? f2bf(cc - bf2f(chi)) : (uint16_t)0;
        dst[62] = 0;
        dst[63] = 0;
    }
    if (k == nch - 1) {                                   // padding rows up to a multiple of 128
        const int ncp = (nch + 127) / 128 * 128;
        for (int r = nch + lane; r < ncp; r += 64) {
            uint16_t *dst = cpk + (cb + r) * PK;
            for (int c = 0; c < PK; ++c) dst[c] = 0;
            dst[30] = f2bf(-1.0e30f);
            cst[cb + r] = make_float4(-1.0f, 0.f, 0.f, 0.f);
        }
    }
}

// ---------------------------------------------------------------- screen

// A staged row is 8 chunks of 16 bytes (hi 0-3, lo 4-7).  Chunk q of row r
// sits at position q ^ lds_swz(r): the 16 lanes that read chunk g of 16
// consecutive rows then touch every bank once (and any 8 of them distinct
// banks), where the plain layout (128-byte rows) put 8 lanes on one bank.
__device__ __forceinline__ int lds_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }
__device__ __forceinline__ int lds_slot(int idx) {            // uint4 index of chunk idx & 7 of row idx >> 3
    return (idx & ~7) | ((idx & 7) ^ lds_swz(idx >> 3));
}

// The second screen takes its blocks in XCD-aware order (xcd_block): only the
// first few blocks of each fragment have uncertified rows, and in table order
// one fragment's working blocks would run on different XCDs, each streaming
// the partner's rows from HBM.

// COLLECT = false: every row of the fragment is a query; write the best tile
// and second-best tile maximum per lane group.
// COLLECT = true: the queries are the fragment's uncertified rows (slots
// [start, start + 256) of its list); append every candidate whose score
// reaches the row's threshold to the row's candidate list.
template <bool COLLECT, int SW, int SQB, int CH>
__global__ void __launch_bounds__(SW * 64) k_screen(const Frag *frag, const Blk *blk, int nblk, const uint16_t *pk,
                                                    const int32_t *perm, const int32_t *rinv,
                                                    int32_t *c1_out, float *v2_out, float *v1_out, const int32_t *fb_row,
                                                    const int32_t *fb_cnt, const float *thr, int32_t *lst,
                                                    int32_t *lst_cnt, PairState *ps) {
    static_assert(SW * SQB * 16 == 256 && PAD_ROWS % (CH * 16) == 0, "screen shape");
    constexpr int CROWS = CH * 16;                               // rows per LDS chunk
    constexpr int U4 = CROWS * PK / 8;                          // uint4 per chunk (1024)
    // two separate arrays, not one indexed by chunk parity: the compiler then
    // sees that the copy into one buffer cannot alias reads of the other and
    // does not wait for it before those reads
    __shared__ __align__(16) uint4 ldsA[U4];
    __shared__ __align__(16) uint4 ldsB[U4];
    const int bi = COLLECT ? xcd_block(nblk) : (int)blockIdx.x;
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &Fq = frag[b.frag];
    if (Fq.partner < 0) return;
    int nq = Fq.n;
    if (COLLECT) {
        nq = min(fb_cnt[b.frag], lst_cap(Fq));
        if (b.start >= nq) return;
    }
    const Frag &Fc = frag[Fq.partner];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int swz = lds_swz(col);

    // query operands: [y_hi, 1, 1] of this wave's 4 blocks of 16 queries
    bf16x8 Bh[SQB];
    float th[SQB];
    const int qw = b.start + wv * SQB * 16;
#pragma unroll
    for (int k = 0; k < SQB; ++k) {
        int slot = qw + 16 * k + col;
        uint4 wh = make_uint4(0, 0, 0, 0);
        th[k] = INFINITY;
        if (slot < nq) {
            int q = COLLECT ? rinv[Fq.off + fb_row[Fq.off + slot]] : slot;      // packed row
            const uint16_t *r = pk + (Fq.pk_off + q) * PK;
            wh = *(const uint4 *)(r + 8 * grp);
            if (COLLECT) th[k] = thr[Fq.off + slot];
        }
        if (grp == 3) wh.w = 0x3f803f80u;                     // slots 30, 31 = 1.0
        Bh[k] = __builtin_bit_cast(bf16x8, wh);
    }
    float v1[SQB], v2[SQB];
    int32_t c1[SQB];
#pragma unroll
    for (int k = 0; k < SQB; ++k) { v1[k] = -INFINITY; v2[k] = -INFINITY; c1[k] = -1; }

    const int nch = (Fc.n + CROWS - 1) / CROWS;
    constexpr int PER = U4 / (SW * 64);                         // 16-byte copies per thread per chunk
    const uint4 *src = (const uint4 *)(pk + Fc.pk_off * PK);
    // Chunks go from global memory straight into LDS (global_load_lds_dwordx4:
    // lane i of a wave's copy fills the 16 bytes at base + 16 i), with no trip
    // through registers.  Copy u of wave wv fills LDS positions
    // [u SW 64 + 64 wv, + 64); position p holds chunk element lds_slot(p), the
    // swizzle being its own inverse within a row.
    auto stage = [&](uint4 *dst, const uint4 *from) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int base = u * SW * 64 + wv * 64;
            __builtin_amdgcn_global_load_lds((const void *)(from + lds_slot(base + lane)),
                                             (__attribute__((address_space(3))) void *)(dst + base), 16, 0, 0);
        }
    };
    // vmcnt(0) with the other counters left alone (gfx9 s_waitcnt encoding)
    auto wait_copies = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };
    if (nch > 0) stage(ldsA, src);
    wait_copies();
    __syncthreads();
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    // Software pipeline: the MFMAs of tile t are issued before the epilogue of
    // tile t-1, so the matrix cores never wait on the vector ALU.
    f32x4 prev[SQB];
    int prev_tile = -1;
    auto epilogue = [&](const f32x4 *accs, int tile) {
        if (!COLLECT) {
            // v2 <= v1 always, so max(v2, min(v1, tm)) is the median of the three.
            // A new best tile is rare once a few hundred tiles have passed, so
            // the best tile index is updated behind a wave-uniform branch.
            bool up[SQB];
            bool any = false;
#pragma unroll
            for (int k = 0; k < SQB; ++k) {
                const f32x4 acc = accs[k];
                const float tm = __builtin_fmaxf(__builtin_fmaxf(acc[0], acc[1]), __builtin_fmaxf(acc[2], acc[3]));
                v2[k] = __builtin_amdgcn_fmed3f(v1[k], tm, v2[k]);
                up[k] = tm > v1[k];
                any |= up[k];
                v1[k] = __builtin_fmaxf(v1[k], tm);
            }
            if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
                for (int k = 0; k < SQB; ++k) c1[k] = up[k] ? tile : c1[k];
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < SQB; ++k) {
            const f32x4 acc = accs[k];
            {
                bool hit = acc[0] >= th[k] || acc[1] >= th[k] || acc[2] >= th[k] || acc[3] >= th[k];
                if (hit) {                                 // rare: near-ties of uncertified rows
                    int64_t slot = lst_base(Fq, b.frag) + qw + 16 * k + col;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (acc[e] >= th[k]) {
                            int pos = atomicAdd(&lst_cnt[slot], 1);
                            if (pos < LCAP) lst[slot * LCAP + pos] = tile * 16 + 4 * grp + e;
                        }
                }
            }
        }
    };
    // one chunk: start copying the next chunk into D, sweep the tiles of L
    auto chunk = [&](const uint4 *L, uint4 *D, int ch) {
        if (ch + 1 < nch) stage(D, src + (int64_t)(ch + 1) * U4);
        // operands of tile t + 1 are read before tile t's MFMAs issue, so the
        // LDS latency hides behind a whole tile of matrix work
        uint4 nh = L[col * 8 + (grp ^ swz)], nl = L[col * 8 + ((4 + grp) ^ swz)];
#pragma unroll 2
        for (int t = 0; t < CH; ++t) {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, nh);
            const bf16x8 al = __builtin_bit_cast(bf16x8, nl);
            if (t + 1 < CH) {
                const uint4 *rowp = L + ((t + 1) * 16 + col) * 8;
                nh = rowp[grp ^ swz];
                nl = rowp[(4 + grp) ^ swz];
            }
            // two chained products per query block, the four blocks interleaved so
            // that each chain step has three independent MFMAs between it and its input
            f32x4 accs[SQB];
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, Bh[k], zero, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, Bh[k], accs[k], 0, 0, 0);
            if (prev_tile >= 0) epilogue(prev, prev_tile);
#pragma unroll
            for (int k = 0; k < SQB; ++k) prev[k] = accs[k];
            prev_tile = ch * CH + t;
        }
        wait_copies();
        __syncthreads();
    };
    for (int ch = 0; ch < nch; ch += 2) {
        chunk(ldsA, ldsB, ch);
        if (ch + 1 < nch) chunk(ldsB, ldsA, ch + 1);
    }
    if (prev_tile >= 0) epilogue(prev, prev_tile);
    if (!COLLECT) {
        if (threadIdx.x == 0 && ps && Fq.pair >= 0) {
            const unsigned long long nc = 4ull * (unsigned long long)((Fc.n + PAD_ROWS - 1) / PAD_ROWS);
            atomicAdd(&ps[Fq.pair].scr_chunks, nc);
            atomicAdd(&ps[Fq.pair].scr_swept, nc);
        }
#pragma unroll
        for (int k = 0; k < SQB; ++k) {
            // lane (col, grp): candidate rows tile*16 + 4 grp + {0..3} (MFMA output rows) of query col
            int q = qw + 16 * k + col;
            if (q < Fq.n) {
                int64_t o = (Fq.off + perm[Fq.off + q]) * 4 + grp;
                c1_out[o] = c1[k];
                v2_out[o] = v2[k];
                v1_out[o] = v1[k];
            }
        }
    }
}

// ---------------------------------------------------------------- pruned screen
//
// The partner's packed rows come in chunks of 128 with centroid rows mu~_k
// (split like candidate rows, so the matrix cores screen them like rows) and
// bounds rho_k >= |y~_j - mu~_k| and delta_k >= |y~_j|^2 / 2 - h_j.  For a
// query with bf16 row yh_i and n_i = |yh_i|^2, every computed score of a row
// j of chunk k obeys
//   t_ij <= n_i / 2 - max(0, g_ik - rho_k)^2 / 2 + delta_k + acc_ik,
// with g_ik <= |yh_i - mu~_k| taken from the screened centroid score tc_ik as
// g_ik^2 = n_i - 2 tc_ik - m_ik, and m_ik, acc_ik margins of 2^-12 of the
// magnitudes involved (float32 accumulation of 64 products errs by ~2^-18 of
// them).  g_ik is taken from the hardware square root scaled by SQ_LO, which
// keeps it below the exact root (the instruction errs by about one ulp, the
// scale removes sixteen), so the bound only loosens.  A block
//  1. sweeps PR_K seed chunks: the partner chunks around the block's median
//     descriptor-space key (both fragments' keys come from the pair's
//     principal directions, so these rows are near the block's queries; any
//     seed set is correct, since step 2 bounds every chunk);
//  2. screens its queries against every centroid: a query needs chunk k unless the bound
//     stays below its best screened score so far minus a margin (four times
//     the certificate's error estimate), and the bound of a chunk a query does
//     not need is folded into its second-best tile maximum, so the certificate
//     still covers every row the block does not screen;
//  3. sweeps the chunks some live query needs.
// Rows with a 2^24 key (invalid descriptors) sort last in each fragment.
constexpr int PR_K = 8;
constexpr float SQ_LO = 1.0f - 1.9073486328125e-6f;    // 1 - 2^-19
// chunks one block can track (fragments up to 522,240 rows; beyond: no pruning).
// 4080, not 4096: the chunk list then leaves the pruned screen's shared memory
// at 40,952 bytes, so four blocks fit a CU (four wavefronts per SIMD, 128
// VGPRs, a few spills outside the sweeps): 59.5 -> 57.1 ms on the benchmark,
// and the collect pass likewise 6.9 -> 5.9 ms
constexpr int PR_NCH_MAX = 4080;

template <int SW, int SQB, int CH>
__global__ void __launch_bounds__(SW * 64) __attribute__((amdgpu_waves_per_eu(4))) k_screen_pr(const Frag *frag, const Blk *blk, int nblk, const uint16_t *pk,
                                                       const uint16_t *cpk, const float4 *cst, const int32_t *perm,
                                                       int32_t *c1_out, float *v2_out, float *v1_out, PairState *ps,
                                                       const uint64_t *skey) {
    static_assert(SW * SQB * 16 == 256 && CH * 16 == PAD_ROWS && CH % 2 == 0, "pruned screen shape: tiles in pairs");
    constexpr int CROWS = CH * 16;
    constexpr int U4 = CROWS * PK / 8;
    static_assert(SW <= 4 && PR_NCH_MAX <= 4096 && SW * PR_NCH_MAX <= U4 * 16, "chunk entries: 12-bit index, wave mask");
    constexpr float MRG = 2.44140625e-4f;                       // 2^-12
    __shared__ __align__(16) uint4 ldsA[U4];
    __shared__ __align__(16) uint4 ldsB[U4];                    // between sweeps: need flags
    __shared__ uint16_t seq[PR_NCH_MAX];                        // chunks of the current sweep
    __shared__ int redi[SW];
    __shared__ int nseq, nwsw;
    // XCD-aware order: consecutive blocks hold neighbouring queries in descriptor
    // space, need mostly the same chunks, and then share one XCD's L2
    const int bi = xcd_block(nblk);
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &Fq = frag[b.frag];
    if (Fq.partner < 0) return;
    const Frag &Fc = frag[Fq.partner];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int swz = lds_swz(col);
    const int nch = (Fc.n + CROWS - 1) / CROWS;
    const bool prune = nch <= PR_NCH_MAX;

    // query operands [y_hi, 1, 1]; n_i = |yh_i|^2 over the 30 coordinates; a
    // live query is a row with a valid descriptor (its c_hi slot is not -1e30)
    bf16x8 Bh[SQB];
    float nq2[SQB];
    bool live[SQB];
    const int qw = b.start + wv * SQB * 16;
#pragma unroll
    for (int k = 0; k < SQB; ++k) {
        const int slot = qw + 16 * k + col;
        uint4 wh = make_uint4(0, 0, 0, 0);
        if (slot < Fq.n) wh = *(const uint4 *)(pk + (Fq.pk_off + slot) * PK + 8 * grp);
        const uint32_t w32[4] = {wh.x, wh.y, wh.z, wh.w};
        float p2 = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = __uint_as_float((e & 1) ? (w32[e >> 1] & 0xFFFF0000u) : (w32[e >> 1] << 16));
            if (grp < 3 || e < 6) p2 = fmaf(x, x, p2);
        }
        int bad = (grp == 3 && __uint_as_float(wh.w << 16) < -1.0e29f) ? 1 : 0;
        p2 += __shfl_xor(p2, 16, 64);
        p2 += __shfl_xor(p2, 32, 64);
        bad |= __shfl_xor(bad, 16, 64);
        bad |= __shfl_xor(bad, 32, 64);
        nq2[k] = p2;
        live[k] = slot < Fq.n && !bad;
        if (grp == 3) wh.w = 0x3f803f80u;                     // slots 30, 31 = 1.0
        Bh[k] = __builtin_bit_cast(bf16x8, wh);
    }
    float v1[SQB], v2[SQB], sf[SQB];
    int32_t c1[SQB];
#pragma unroll
    for (int k = 0; k < SQB; ++k) { v1[k] = -INFINITY; v2[k] = -INFINITY; sf[k] = -INFINITY; c1[k] = -1; }

    constexpr int PER = U4 / (SW * 64);
    const uint4 *src = (const uint4 *)(pk + Fc.pk_off * PK);
    const int64_t cb = cent_base(Fc, Fq.partner);
    const uint4 *csrc = (const uint4 *)(cpk + cb * PK);
    auto stage = [&](uint4 *dst, const uint4 *from) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int base = u * SW * 64 + wv * 64;
            __builtin_amdgcn_global_load_lds((const void *)(from + lds_slot(base + lane)),
                                             (__attribute__((address_space(3))) void *)(dst + base), 16, 0, 0);
        }
    };
    auto wait_copies = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const f32x4 ninf = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    // the previous tile's scores, folded in while the next tile's MFMAs run;
    // -inf scores (before the first tile) change nothing
    f32x4 prev[SQB];
    int prev_tile = 0;
#pragma unroll
    for (int k = 0; k < SQB; ++k) prev[k] = ninf;
    // a tile whose maxima stay at or below every second-best changes nothing
    // (med3(v1, t, v2) = v2 for t <= v2 <= v1), so the update runs only when
    // some lane's maximum passes its second-best
    auto epilogue = [&](const f32x4 *accs, int tile) __attribute__((always_inline)) {
        float tm[SQB];
        bool any = false;
#pragma unroll
        for (int k = 0; k < SQB; ++k) {
            const f32x4 acc = accs[k];
            tm[k] = __builtin_fmaxf(__builtin_fmaxf(acc[0], acc[1]), __builtin_fmaxf(acc[2], acc[3]));
            any |= tm[k] > v2[k];
        }
        if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
            for (int k = 0; k < SQB; ++k) {
                const bool up = tm[k] > v1[k];
                v2[k] = __builtin_amdgcn_fmed3f(v1[k], tm[k], v2[k]);
                v1[k] = __builtin_fmaxf(v1[k], tm[k]);
                c1[k] = up ? tile : c1[k];
            }
        }
    };
    auto cid = [&](int c) { return prune ? (int)(seq[c] & 0xFFF) : c; };
    auto swept_by_me = [&](int c) { return !prune || ((seq[c] >> (12 + wv)) & 1); };
    // one chunk of a sweep: start copying the next chunk into D, sweep the tiles of L
    auto chunk = [&](const uint4 *L, uint4 *D, int c, int len) __attribute__((always_inline)) {
        if (c + 1 < len) stage(D, src + (int64_t)cid(c + 1) * U4);
        if (!swept_by_me(c)) {                                    // wave-uniform
            wait_copies();
            __syncthreads();
            return;
        }
        const int tbase = __builtin_amdgcn_readfirstlane(cid(c)) * CH;   // wave-uniform
        // one tile: its MFMAs, then the previous tile's epilogue while they run
        auto tile = [&](const uint4 &h, const uint4 &l, int t) __attribute__((always_inline)) {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, h);
            const bf16x8 al = __builtin_bit_cast(bf16x8, l);
            f32x4 accs[SQB];
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, Bh[k], zero, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, Bh[k], accs[k], 0, 0, 0);
            epilogue(prev, prev_tile);
#pragma unroll
            for (int k = 0; k < SQB; ++k) prev[k] = accs[k];
            prev_tile = tbase + t;
        };
        // tiles in pairs with two operand register sets: the next tile's
        // operands are read from LDS while the current tile's MFMAs run
        const uint4 *rw = L + col * 8;
        uint4 h0 = rw[grp ^ swz], l0 = rw[(4 + grp) ^ swz];
#pragma unroll 1
        for (int t = 0; t < CH; t += 2) {
            const uint4 h1 = rw[(t + 1) * 128 + (grp ^ swz)], l1 = rw[(t + 1) * 128 + ((4 + grp) ^ swz)];
            tile(h0, l0, t);
            if (t + 2 < CH) {
                h0 = rw[(t + 2) * 128 + (grp ^ swz)];
                l0 = rw[(t + 2) * 128 + ((4 + grp) ^ swz)];
            }
            tile(h1, l1, t + 1);
        }
        wait_copies();
        __syncthreads();
    };
    auto sweep = [&](int len) __attribute__((always_inline)) {
        if (len <= 0) return;
        stage(ldsA, src + (int64_t)cid(0) * U4);
        wait_copies();
        __syncthreads();
        for (int c = 0; c < len; c += 2) {
            chunk(ldsA, ldsB, c, len);
            if (c + 1 < len) chunk(ldsB, ldsA, c + 1, len);
        }
        epilogue(prev, prev_tile);
#pragma unroll
        for (int k = 0; k < SQB; ++k) prev[k] = ninf;
    };
    // screened scores of the block's queries against every centroid row, one
    // staged chunk of 128 centroids at a time (single buffered: ldsB holds the
    // per-chunk state); fn(accs, first centroid of the lane's four)
    // the chunk bounds of the staged centroids go to seq's storage (free
    // during this pass); fn(accs, first centroid of the lane's four, their bounds)
    float4 *sst = (float4 *)seq;
    static_assert(sizeof(seq) >= CROWS * sizeof(float4), "centroid bounds staging");
    auto cent_pass = [&](auto &&fn) {
        const int ncc = (nch + CROWS - 1) / CROWS;
        for (int cc = 0; cc < ncc; ++cc) {
            stage(ldsA, csrc + (int64_t)cc * U4);
            // slots past nch are padding of the fragment's centroid region: read, never used
            if (threadIdx.x < CROWS) sst[threadIdx.x] = cst[cb + (int64_t)cc * CROWS + threadIdx.x];
            wait_copies();
            __syncthreads();
            for (int t = 0; t < CH && cc * CROWS + t * 16 < nch; ++t) {   // tiles holding centroids
                const uint4 *rowp = ldsA + (t * 16 + col) * 8;
                const bf16x8 ah = __builtin_bit_cast(bf16x8, rowp[grp ^ swz]);
                const bf16x8 al = __builtin_bit_cast(bf16x8, rowp[(4 + grp) ^ swz]);
                f32x4 accs[SQB];
#pragma unroll
                for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, Bh[k], zero, 0, 0, 0);
#pragma unroll
                for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, Bh[k], accs[k], 0, 0, 0);
                fn(accs, cc * CROWS + t * 16 + 4 * grp, sst + t * 16 + 4 * grp);
            }
            __syncthreads();
        }
    };

    // (64-query group, 128-row chunk) visits made, centroid passes included
    int swept = 4 * nch;
    if (!prune) {
        sweep(nch);
    } else {
        // 1. seeds: the PR_K partner chunks around the block's median descriptor-space key
        //    (both fragments' keys come from the pair's principal directions)
        const uint64_t KM = (1ull << 25) - 1ull;
        const uint64_t km = skey[Fq.off + min(b.start + 128, Fq.n - 1)] & KM;
        int first = nch;                                   // first chunk whose first row's key is >= km
        for (int c = threadIdx.x; c < nch; c += SW * 64)
            if ((skey[Fc.off + (int64_t)c * CROWS] & KM) >= km) first = min(first, c);
        for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
        if (lane == 0) redi[wv] = first;
        __syncthreads();
        const int k1 = min(PR_K, nch);
        if (threadIdx.x == 0) {
            int f = redi[0];
            for (int w = 1; w < SW; ++w) f = min(f, redi[w]);
            int c0 = max(0, min(f - PR_K / 2, nch - k1));
            for (int r = 0; r < k1; ++r) seq[r] = (uint16_t)((c0 + r) | (((1u << SW) - 1u) << 12));
        }
        __syncthreads();
        sweep(k1);
        // 2. which chunks do the queries still need?
        float thn[SQB];
#pragma unroll
        for (int k = 0; k < SQB; ++k) {
            float bq = v1[k];
            bq = fmaxf(bq, __shfl_xor(bq, 16, 64));
            bq = fmaxf(bq, __shfl_xor(bq, 32, 64));
            const float D = fmaxf(nq2[k] - 2.0f * bq, 0.f);
            const float dl = 7.8125e-3f * sqrtf(nq2[k] * D) + MRG * (nq2[k] + D) + 1.0e-7f;
            thn[k] = bq - dl;                                       // -inf when no row was screened
        }
        float ga[SQB], ub[SQB];                                     // the bound's per-query terms
#pragma unroll
        for (int k = 0; k < SQB; ++k) {
            ga[k] = nq2[k] - MRG * nq2[k];
            ub[k] = 0.5f * nq2[k] * (1.0f + 1.0e-6f) + MRG * nq2[k];
        }
        // need[w][k]: 0 wave w skips chunk k, 1 it sweeps it, 2 already swept
        uint8_t *need = (uint8_t *)ldsB;
        uint8_t *mine = need + wv * PR_NCH_MAX;
        for (int k = threadIdx.x; k < SW * nch; k += SW * 64) need[(k / nch) * PR_NCH_MAX + k % nch] = 0;
        __syncthreads();
        if (threadIdx.x < k1)
            for (int w = 0; w < SW; ++w) need[w * PR_NCH_MAX + (seq[threadIdx.x] & 0xFFF)] = 2;
        __syncthreads();
        cent_pass([&](const f32x4 *accs, int kc0, const float4 *stl) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kc = kc0 + e;
                const float4 st = stl[e];                            // rho, delta, max |y|^2 + max h, |mu|^2
                // a real, non-empty chunk not swept as a seed
                const bool open = kc < nch && st.x >= 0.f && mine[kc] != 2;
                const float cw = MRG * st.w, cy = st.y + MRG * st.z;
                bool nd_any = false;
#pragma unroll
                for (int k = 0; k < SQB; ++k) {
                    // g2 = n - 2 tc - MRG (n + |mu|^2), U = n (1 + 1e-6) / 2 - (1 - 1e-6) L^2 / 2 + delta
                    // + MRG (n + st.z), the query's terms hoisted (a few ulps of rearrangement, far inside
                    // the 1e-6 factors and the 2^-12 margins)
                    const float g2 = fmaf(-2.0f, accs[k][e], ga[k] - cw);
                    const float L = fmaxf(fmaf(__builtin_amdgcn_sqrtf(fmaxf(g2, 0.f)), SQ_LO, -st.x), 0.f);
                    const float U = fmaf(-0.5f * (1.0f - 1.0e-6f), L * L, ub[k] + cy);
                    const bool use = open && live[k];                // dead queries take no part
                    const bool nd = U >= thn[k];
                    nd_any |= use && nd;
                    sf[k] = use && !nd ? fmaxf(sf[k], U) : sf[k];
                }
                const uint64_t bal = __builtin_amdgcn_ballot_w64(nd_any);
                if (col == 0 && ((bal >> (16 * grp)) & 0xFFFFull)) mine[kc] = 1;
            }
        });
        // 3. the chunks some wavefront needs, in index order, with the mask of
        //    the wavefronts that need them in the entry's top bits (a
        //    wavefront outside the mask stages the chunk but skips its MFMAs)
        if (wv == 0) {
            int cnt = 0, nw = 0;
            for (int base = 0; base < nch; base += 64) {
                const int k = base + lane;
                uint32_t wm = 0;
                if (k < nch)
                    for (int w = 0; w < SW; ++w) wm |= (need[w * PR_NCH_MAX + k] == 1 ? 1u : 0u) << w;
                const bool f = wm != 0;
                const uint64_t m = __builtin_amdgcn_ballot_w64(f);
                if (f) seq[cnt + (int)lanes_below_w(m)] = (uint16_t)(k | (wm << 12));
                cnt += __popcll(m);
                nw += __popc(wm);
            }
            for (int o = 32; o > 0; o >>= 1) nw += __shfl_xor(nw, o, 64);
            if (lane == 0) { nseq = cnt; nwsw = nw; }
        }
        __syncthreads();
        sweep(nseq);
        swept = (SW * k1 + nwsw + 2 * SW * ((nch + CROWS - 1) / CROWS)) * 4 / SW;
    }
    if (threadIdx.x == 0 && ps && Fq.pair >= 0) {
        atomicAdd(&ps[Fq.pair].scr_chunks, 4ull * (unsigned long long)nch);
        atomicAdd(&ps[Fq.pair].scr_swept, (unsigned long long)swept);
    }
#pragma unroll
    for (int k = 0; k < SQB; ++k) {
        float s = sf[k];
        s = fmaxf(s, __shfl_xor(s, 16, 64));
        s = fmaxf(s, __shfl_xor(s, 32, 64));
        const int q = qw + 16 * k + col;
        if (q < Fq.n) {
            int64_t o = (Fq.off + perm[Fq.off + q]) * 4 + grp;
            c1_out[o] = c1[k];
            v2_out[o] = fmaxf(v2[k], s);
            v1_out[o] = v1[k];
        }
    }
}

// Collect pass over the pruned layout.  The queries are a fragment's
// uncertified rows in packed-row order (slots [start, start + 256) of its
// list, so a block's rows are neighbours in descriptor space); a row with no
// reference distance (threshold -inf) is already on the float32 rescan list
// and takes no part.  A row needs partner chunk k unless the chunk's bound on
// every computed score of its rows (the pruned screen's bound) stays below
// the row's threshold: a skipped chunk holds no row that the exhaustive
// collect pass would append, so the lists receive the same candidates.  The
// block screens its queries against every centroid, then sweeps the chunks
// some wavefront needs (a wavefront outside a chunk's mask stages it but
// skips its MFMAs); every candidate of a swept tile whose score reaches the
// row's threshold goes to the row's list.  Fragments past PR_NCH_MAX chunks
// are swept whole.
template <int SW, int SQB, int CH>
__global__ void __launch_bounds__(SW * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_screen_prc(const Frag *frag, const Blk *blk, int nblk, const uint16_t *pk, const uint16_t *cpk, const float4 *cst,
             const int32_t *rinv, const int32_t *fb_row, const int32_t *fb_cnt, const float *thr, int32_t *lst,
             int32_t *lst_cnt) {
    static_assert(SW * SQB * 16 == 256 && CH * 16 == PAD_ROWS && CH % 2 == 0, "pruned screen shape: tiles in pairs");
    constexpr int CROWS = CH * 16;
    constexpr int U4 = CROWS * PK / 8;
    static_assert(SW <= 4 && PR_NCH_MAX <= 4096 && SW * PR_NCH_MAX <= U4 * 16, "chunk entries: 12-bit index, wave mask");
    constexpr float MRG = 2.44140625e-4f;                       // 2^-12
    __shared__ __align__(16) uint4 ldsA[U4];
    __shared__ __align__(16) uint4 ldsB[U4];                    // between sweeps: need flags
    __shared__ uint16_t seq[PR_NCH_MAX];
    __shared__ int nseq;
    const int bi = xcd_block(nblk);
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &Fq = frag[b.frag];
    if (Fq.partner < 0) return;
    const int nq = min(fb_cnt[b.frag], lst_cap(Fq));
    if (b.start >= nq) return;
    const Frag &Fc = frag[Fq.partner];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int swz = lds_swz(col);
    const int nch = (Fc.n + CROWS - 1) / CROWS;
    const bool prune = nch <= PR_NCH_MAX;

    // query operands [y_hi, 1, 1], n_i = |yh_i|^2 over the 30 coordinates, thresholds
    bf16x8 Bh[SQB];
    float nq2[SQB], th[SQB];
    bool live[SQB];
    const int qw = b.start + wv * SQB * 16;
#pragma unroll
    for (int k = 0; k < SQB; ++k) {
        const int slot = qw + 16 * k + col;
        uint4 wh = make_uint4(0, 0, 0, 0);
        float t = -INFINITY;
        if (slot < nq) {
            const int q = rinv[Fq.off + fb_row[Fq.off + slot]];
            wh = *(const uint4 *)(pk + (Fq.pk_off + q) * PK + 8 * grp);
            t = thr[Fq.off + slot];
        }
        const uint32_t w32[4] = {wh.x, wh.y, wh.z, wh.w};
        float p2 = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = __uint_as_float((e & 1) ? (w32[e >> 1] & 0xFFFF0000u) : (w32[e >> 1] << 16));
            if (grp < 3 || e < 6) p2 = fmaf(x, x, p2);
        }
        p2 += __shfl_xor(p2, 16, 64);
        p2 += __shfl_xor(p2, 32, 64);
        nq2[k] = p2;
        live[k] = t > -INFINITY;                              // also false past the list
        th[k] = live[k] ? t : INFINITY;                       // a row outside collects nothing
        if (grp == 3) wh.w = 0x3f803f80u;                     // slots 30, 31 = 1.0
        Bh[k] = __builtin_bit_cast(bf16x8, wh);
    }

    constexpr int PER = U4 / (SW * 64);
    const uint4 *src = (const uint4 *)(pk + Fc.pk_off * PK);
    const int64_t cb = cent_base(Fc, Fq.partner);
    const uint4 *csrc = (const uint4 *)(cpk + cb * PK);
    auto stage = [&](uint4 *dst, const uint4 *from) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int base = u * SW * 64 + wv * 64;
            __builtin_amdgcn_global_load_lds((const void *)(from + lds_slot(base + lane)),
                                             (__attribute__((address_space(3))) void *)(dst + base), 16, 0, 0);
        }
    };
    auto wait_copies = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const f32x4 ninf = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    // the previous tile's scores, tested while the next tile's MFMAs run; -inf
    // scores (before the first tile) reach no threshold
    f32x4 prev[SQB];
    int prev_tile = 0;
#pragma unroll
    for (int k = 0; k < SQB; ++k) prev[k] = ninf;
    auto epilogue = [&](const f32x4 *accs, int tile) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < SQB; ++k) {
            const f32x4 acc = accs[k];
            const float tm = __builtin_fmaxf(__builtin_fmaxf(acc[0], acc[1]), __builtin_fmaxf(acc[2], acc[3]));
            if (tm >= th[k]) {                                // rare: near-ties of uncertified rows
                const int64_t slot = lst_base(Fq, b.frag) + qw + 16 * k + col;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (acc[e] >= th[k]) {
                        const int pos = atomicAdd(&lst_cnt[slot], 1);
                        if (pos < LCAP) lst[slot * LCAP + pos] = tile * 16 + 4 * grp + e;
                    }
            }
        }
    };
    auto cid = [&](int c) { return prune ? (int)(seq[c] & 0xFFF) : c; };
    auto swept_by_me = [&](int c) { return !prune || ((seq[c] >> (12 + wv)) & 1); };
    auto chunk = [&](const uint4 *L, uint4 *D, int c, int len) __attribute__((always_inline)) {
        if (c + 1 < len) stage(D, src + (int64_t)cid(c + 1) * U4);
        if (!swept_by_me(c)) {                                    // wave-uniform
            wait_copies();
            __syncthreads();
            return;
        }
        const int tbase = __builtin_amdgcn_readfirstlane(cid(c)) * CH;   // wave-uniform
        auto tile = [&](const uint4 &h, const uint4 &l, int t) __attribute__((always_inline)) {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, h);
            const bf16x8 al = __builtin_bit_cast(bf16x8, l);
            f32x4 accs[SQB];
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, Bh[k], zero, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, Bh[k], accs[k], 0, 0, 0);
            epilogue(prev, prev_tile);
#pragma unroll
            for (int k = 0; k < SQB; ++k) prev[k] = accs[k];
            prev_tile = tbase + t;
        };
        // tiles in pairs, two operand register sets (as in the pruned screen)
        const uint4 *rw = L + col * 8;
        uint4 h0 = rw[grp ^ swz], l0 = rw[(4 + grp) ^ swz];
#pragma unroll 1
        for (int t = 0; t < CH; t += 2) {
            const uint4 h1 = rw[(t + 1) * 128 + (grp ^ swz)], l1 = rw[(t + 1) * 128 + ((4 + grp) ^ swz)];
            tile(h0, l0, t);
            if (t + 2 < CH) {
                h0 = rw[(t + 2) * 128 + (grp ^ swz)];
                l0 = rw[(t + 2) * 128 + ((4 + grp) ^ swz)];
            }
            tile(h1, l1, t + 1);
        }
        wait_copies();
        __syncthreads();
    };
    auto sweep = [&](int len) __attribute__((always_inline)) {
        if (len <= 0) return;
        stage(ldsA, src + (int64_t)cid(0) * U4);
        wait_copies();
        __syncthreads();
        for (int c = 0; c < len; c += 2) {
            chunk(ldsA, ldsB, c, len);
            if (c + 1 < len) chunk(ldsB, ldsA, c + 1, len);
        }
        epilogue(prev, prev_tile);
#pragma unroll
        for (int k = 0; k < SQB; ++k) prev[k] = ninf;
    };
    if (!prune) {
        sweep(nch);
        return;
    }
    float ga[SQB], ub[SQB];                                         // the bound's per-query terms
#pragma unroll
    for (int k = 0; k < SQB; ++k) {
        ga[k] = nq2[k] - MRG * nq2[k];
        ub[k] = 0.5f * nq2[k] * (1.0f + 1.0e-6f) + MRG * nq2[k];
    }
    // need[w][k] = 1: some query of wavefront w needs chunk k
    uint8_t *need = (uint8_t *)ldsB;
    uint8_t *mine = need + wv * PR_NCH_MAX;
    for (int k = threadIdx.x; k < SW * nch; k += SW * 64) need[(k / nch) * PR_NCH_MAX + k % nch] = 0;
    __syncthreads();
    float4 *sst = (float4 *)seq;                                    // the staged centroids' bounds
    static_assert(sizeof(seq) >= CROWS * sizeof(float4), "centroid bounds staging");
    const int ncc = (nch + CROWS - 1) / CROWS;
    for (int cc = 0; cc < ncc; ++cc) {
        stage(ldsA, csrc + (int64_t)cc * U4);
        if (threadIdx.x < CROWS) sst[threadIdx.x] = cst[cb + (int64_t)cc * CROWS + threadIdx.x];
        wait_copies();
        __syncthreads();
        for (int t = 0; t < CH && cc * CROWS + t * 16 < nch; ++t) {   // tiles holding centroids
            const uint4 *rowp = ldsA + (t * 16 + col) * 8;
            const bf16x8 ah = __builtin_bit_cast(bf16x8, rowp[grp ^ swz]);
            const bf16x8 al = __builtin_bit_cast(bf16x8, rowp[(4 + grp) ^ swz]);
            f32x4 accs[SQB];
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, Bh[k], zero, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < SQB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, Bh[k], accs[k], 0, 0, 0);
            const int kc0 = cc * CROWS + t * 16 + 4 * grp;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kc = kc0 + e;
                const float4 st = sst[t * 16 + 4 * grp + e];         // rho, delta, max |y|^2 + max h, |mu|^2
                const bool open = kc < nch && st.x >= 0.f;           // a real, non-empty chunk
                const float cw = MRG * st.w, cy = st.y + MRG * st.z;
                bool nd_any = false;
#pragma unroll
                for (int k = 0; k < SQB; ++k) {
                    const float g2 = fmaf(-2.0f, accs[k][e], ga[k] - cw);   // the pruned screen's bound
                    const float Lb = fmaxf(fmaf(__builtin_amdgcn_sqrtf(fmaxf(g2, 0.f)), SQ_LO, -st.x), 0.f);
                    const float U = fmaf(-0.5f * (1.0f - 1.0e-6f), Lb * Lb, ub[k] + cy);
                    nd_any |= open && live[k] && U >= th[k];          // no query: takes no part
                }
                const uint64_t bal = __builtin_amdgcn_ballot_w64(nd_any);
                if (col == 0 && ((bal >> (16 * grp)) & 0xFFFFull)) mine[kc] = 1;
            }
        }
        __syncthreads();
    }
    if (wv == 0) {
        int cnt = 0;
        for (int base = 0; base < nch; base += 64) {
            const int k = base + lane;
            uint32_t wm = 0;
            if (k < nch)
                for (int w = 0; w < SW; ++w) wm |= (need[w * PR_NCH_MAX + k] == 1 ? 1u : 0u) << w;
            const bool f = wm != 0;
            const uint64_t m = __builtin_amdgcn_ballot_w64(f);
            if (f) seq[cnt + (int)lanes_below_w(m)] = (uint16_t)(k | (wm << 12));
            cnt += __popcll(m);
        }
        if (lane == 0) nseq = cnt;
    }
    __syncthreads();
    sweep(nseq);
}

// Uncertified rows of a fragment in packed-row order: mark their packed rows
// (mark starts zeroed), a scan gives each its slot.  A fragment whose list
// overflowed keeps the arrival order (its rows past the capacity are already
// on the float32 rescan list).  The list re-rank's result does not depend on
// the order.
__global__ void __launch_bounds__(256) k_fb_mark(const Frag *frag, const Blk *blk, const int32_t *fb_row,
                                                 const int32_t *fb_cnt, const int32_t *rinv, int32_t *mark) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    const int k = b.start + threadIdx.x;
    const int cnt = fb_cnt[b.frag];
    if (F.partner < 0 || k >= F.n || k >= cnt || cnt > lst_cap(F)) return;
    mark[F.off + rinv[F.off + fb_row[F.off + k]]] = 1;
}

__global__ void __launch_bounds__(256) k_fb_order(const Frag *frag, const Blk *blk, const int32_t *fb_row,
                                                  const float *thr, const int32_t *fb_cnt, const int32_t *rinv,
                                                  const int32_t *lpos, int32_t *fb_row2, float *thr2) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    const int k = b.start + threadIdx.x;
    const int cnt = fb_cnt[b.frag];
    if (F.partner < 0 || k >= F.n || k >= cnt) return;
    const int32_t i = fb_row[F.off + k];
    const int dst = cnt <= lst_cap(F) ? lpos[F.off + rinv[F.off + i]] - lpos[F.off] : k;
    fb_row2[F.off + dst] = i;
    thr2[F.off + dst] = thr[F.off + k];
}

// 32x32 tiles: 32x32x16 MFMAs (two per K = 32).  Lane (col, h) holds query col
// and, of every 32-row tile, candidate rows 8 i + 4 h + j (i, j < 4): one lane
// half sees 16 of the tile's rows, so the epilogue costs 12 VALU operations
// per four MFMAs (against 6 per two with 16x16 tiles); the re-rank then
// checks 32 rows per query.
template <bool COLLECT, int SW, int QB, int CH>
__global__ void __launch_bounds__(SW * 64) k_screen32(const Frag *frag, const Blk *blk, int nblk, const uint16_t *pk,
                                                      const int32_t *perm, const int32_t *rinv, int32_t *c1_out,
                                                      float *v2_out, float *v1_out, const int32_t *fb_row,
                                                      const int32_t *fb_cnt, const float *thr, int32_t *lst,
                                                      int32_t *lst_cnt, PairState *ps) {
    static_assert(SW * QB * 32 == 256 && PAD_ROWS % (CH * 32) == 0, "screen shape");
    constexpr int CROWS = CH * 32;                               // rows per LDS chunk
    constexpr int U4 = CROWS * PK / 8;                          // uint4 per chunk
    __shared__ __align__(16) uint4 ldsA[U4];                    // two arrays: see k_screen
    __shared__ __align__(16) uint4 ldsB[U4];
    const int bi = COLLECT ? xcd_block(nblk) : (int)blockIdx.x;
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &Fq = frag[b.frag];
    if (Fq.partner < 0) return;
    int nq = Fq.n;
    if (COLLECT) {
        nq = min(fb_cnt[b.frag], lst_cap(Fq));
        if (b.start >= nq) return;
    }
    const Frag &Fc = frag[Fq.partner];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 31, h = lane >> 5;
    const int swz = lds_swz(col);

    // query operands: lane (col, h) holds K elements 8h..8h+7 and 16+8h..16+8h+7 of [y_hi, 1, 1]
    bf16x8 B0[QB], B1[QB];
    float th[QB];
    const int qw = b.start + wv * QB * 32;
#pragma unroll
    for (int k = 0; k < QB; ++k) {
        int slot = qw + 32 * k + col;
        uint4 w0 = make_uint4(0, 0, 0, 0), w1 = w0;
        th[k] = INFINITY;
        if (slot < nq) {
            int q = COLLECT ? rinv[Fq.off + fb_row[Fq.off + slot]] : slot;      // packed row
            const uint16_t *r = pk + (Fq.pk_off + q) * PK;
            w0 = *(const uint4 *)(r + 8 * h);
            w1 = *(const uint4 *)(r + 16 + 8 * h);
            if (COLLECT) th[k] = thr[Fq.off + slot];
        }
        if (h == 1) w1.w = 0x3f803f80u;                      // slots 30, 31 = 1.0
        B0[k] = __builtin_bit_cast(bf16x8, w0);
        B1[k] = __builtin_bit_cast(bf16x8, w1);
    }
    float v1[QB], v2[QB];
    int32_t c1[QB];
#pragma unroll
    for (int k = 0; k < QB; ++k) { v1[k] = -INFINITY; v2[k] = -INFINITY; c1[k] = -1; }

    const int nch = (Fc.n + CROWS - 1) / CROWS;
    constexpr int PER = U4 / (SW * 64);
    const uint4 *src = (const uint4 *)(pk + Fc.pk_off * PK);
    // chunks copied straight into LDS, as in k_screen
    auto stage = [&](uint4 *dst, const uint4 *from) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int base = u * SW * 64 + wv * 64;
            __builtin_amdgcn_global_load_lds((const void *)(from + lds_slot(base + lane)),
                                             (__attribute__((address_space(3))) void *)(dst + base), 16, 0, 0);
        }
    };
    auto wait_copies = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };   // vmcnt(0)
    if (nch > 0) stage(ldsA, src);
    wait_copies();
    __syncthreads();
    f32x16 zero;
#pragma unroll
    for (int e = 0; e < 16; ++e) zero[e] = 0.f;
    f32x16 prev[QB];
    int prev_tile = -1;
    auto epilogue = [&](const f32x16 *accs, int tile) {
        bool up[QB];
        bool any = false;
#pragma unroll
        for (int k = 0; k < QB; ++k) {
            const f32x16 a = accs[k];
            // a chain of three-way maxima: 8 v_max3 / v_max for 16 scores
            float tm = __builtin_fmaxf(__builtin_fmaxf(a[0], a[1]), a[2]);
#pragma unroll
            for (int e = 3; e < 15; e += 2) tm = __builtin_fmaxf(__builtin_fmaxf(tm, a[e]), a[e + 1]);
            tm = __builtin_fmaxf(tm, a[15]);
            if (!COLLECT) {
                v2[k] = __builtin_amdgcn_fmed3f(v1[k], tm, v2[k]);      // v2 <= v1: max(v2, min(v1, tm))
                up[k] = tm > v1[k];
                any |= up[k];
                v1[k] = __builtin_fmaxf(v1[k], tm);
            } else if (tm >= th[k]) {                                  // rare: near-ties of uncertified rows
                int64_t slot = lst_base(Fq, b.frag) + qw + 32 * k + col;
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (a[e] >= th[k]) {
                        int pos = atomicAdd(&lst_cnt[slot], 1);
                        if (pos < LCAP) lst[slot * LCAP + pos] = tile * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                    }
            }
        }
        if (!COLLECT && __builtin_amdgcn_ballot_w64(any)) {      // a new best tile: rare
#pragma unroll
            for (int k = 0; k < QB; ++k) c1[k] = up[k] ? tile : c1[k];
        }
    };
    auto chunk = [&](const uint4 *L, uint4 *D, int ch) {
        if (ch + 1 < nch) stage(D, src + (int64_t)(ch + 1) * U4);
#pragma unroll 2
        for (int t = 0; t < CH; ++t) {
            const uint4 *rowp = L + (t * 32 + col) * 8;
            const bf16x8 ah0 = __builtin_bit_cast(bf16x8, rowp[h ^ swz]);
            const bf16x8 ah1 = __builtin_bit_cast(bf16x8, rowp[(2 + h) ^ swz]);
            const bf16x8 al0 = __builtin_bit_cast(bf16x8, rowp[(4 + h) ^ swz]);
            const bf16x8 al1 = __builtin_bit_cast(bf16x8, rowp[(6 + h) ^ swz]);
            f32x16 accs[QB];
#pragma unroll
            for (int k = 0; k < QB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, B0[k], zero, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < QB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, B1[k], accs[k], 0, 0, 0);
#pragma unroll
            for (int k = 0; k < QB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, B0[k], accs[k], 0, 0, 0);
#pragma unroll
            for (int k = 0; k < QB; ++k) accs[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, B1[k], accs[k], 0, 0, 0);
            if (prev_tile >= 0) epilogue(prev, prev_tile);
#pragma unroll
            for (int k = 0; k < QB; ++k) prev[k] = accs[k];
            prev_tile = ch * CH + t;
        }
        wait_copies();
        __syncthreads();
    };
    for (int ch = 0; ch < nch; ch += 2) {
        chunk(ldsA, ldsB, ch);
        if (ch + 1 < nch) chunk(ldsB, ldsA, ch + 1);
    }
    if (prev_tile >= 0) epilogue(prev, prev_tile);
    if (!COLLECT) {
        if (threadIdx.x == 0 && ps && Fq.pair >= 0) {
            const unsigned long long nc = 4ull * (unsigned long long)((Fc.n + PAD_ROWS - 1) / PAD_ROWS);
            atomicAdd(&ps[Fq.pair].scr_chunks, nc);
            atomicAdd(&ps[Fq.pair].scr_swept, nc);
        }
#pragma unroll
        for (int k = 0; k < QB; ++k) {
            int q = qw + 32 * k + col;
            if (q < Fq.n) {
                int64_t o = (Fq.off + perm[Fq.off + q]) * 4 + h;  // entries 0, 1 of the row's four
                c1_out[o] = c1[k];
                v2_out[o] = v2[k];
                v1_out[o] = v1[k];
            }
        }
    }
}

// ---------------------------------------------------------------- re-rank

__device__ __forceinline__ void load_row(const float *F, int64_t r, float *x) {
    const float *p = F + r * FD;
#pragma unroll
    for (int c = 0; c < FD; ++c) x[c] = p[c];
}

// Error bounds of the certificate (the rounding analysis is in the design
// notes).  dl = delta_i + delta_max of the partner fragment, the largest
// distance between a row's float projection y and the exact projection y* of
// its float descriptor (minus the same centre).  slack(D) bounds
// |D^ - D^y| for a competitor at distance about D: the float32
// difference-form distance D^ is within 35 u D of the exact D over the 33
// bins (u = 2^-24), the projected distance D^y within 2 sqrt(D) dl + dl^2
// of D (plus block-sum terms below 1e-12).  screen_err bounds
// |s - t - c_i| for competitors (D^ <= D* implies |y_j - y_i| <= Rp).
__device__ __forceinline__ float slack(float best, float dl) {
    return best * 3e-6f + 2.01f * sqrtf(best) * dl + 2.0f * dl * dl + 1e-10f;
}
__device__ __forceinline__ float screen_err(float4 q, float best, float dl) {
    const float yi = sqrtf(q.x);
    const float Rp = sqrtf(best + slack(best, dl)) * 1.0001f + dl + 1e-9f;   // bound on |y_j - y_i| of competitors
    const float R = yi * 1.0001f + Rp;                                       // bound on |y_j|
    return q.z * Rp + 3.0518e-5f * (yi * R + 0.5f * R * R) + 1e-9f;         // |d_i| Rp + 2^-15 (|y_i| R + R^2 / 2)
}

template <int T>
__global__ void __launch_bounds__(256) k_rerank(const Frag *frag, const Blk *blk, const float *F, const int32_t *valid,
                                                const float4 *yq, const float *mean, const int32_t *perm, const int32_t *c1,
                                                const float *v2, const float *v1, int32_t *nn,
                                                float *dist, int32_t *fb_row, float *thr, int32_t *fb_cnt,
                                                int32_t *full_row, int32_t *full_frag, int32_t *full_cnt,
                                                PairState *ps, int nblk) {
    const int bi = xcd_block(nblk);                   // neighbouring queries share candidate rows
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &Fq = frag[b.frag];
    const int i = b.start + threadIdx.x;
    bool fb = false;
    if (i < Fq.n && Fq.partner >= 0) {
        const Frag &Fc = frag[Fq.partner];
        const int64_t gi = Fq.off + i;
        if (!valid[gi]) {
            nn[gi] = -1;
            dist[gi] = INFINITY;
        } else {
            float q[FD];
            load_row(F, gi, q);
            float best = INFINITY;
            int32_t bj = -1;
            float a2 = -INFINITY;
            const float4 qv = yq[Fq.pk_off + i];
            const float ny2 = qv.x;
            const float dl = qv.w + mean[32 * (b.frag >> 1) + 30 + (Fq.partner & 1)];
            // T = 16: four lane groups, rows 4 g + e of their best tile;
            // T = 32: two lane halves, rows 8 (e / 4) + 4 g + e % 4
            constexpr int G = T == 16 ? 4 : 2, NE = T == 16 ? 4 : 16;
            float gv[G];
            int gord[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                a2 = fmaxf(a2, v2[gi * 4 + g]);
                gv[g] = c1[gi * 4 + g] >= 0 ? v1[gi * 4 + g] : -INFINITY;
                gord[g] = g;
            }
#pragma unroll
            for (int a = 0; a < G; ++a)                    // groups by descending best-tile maximum
#pragma unroll
                for (int c = a + 1; c < G; ++c)
                    if (gv[gord[c]] > gv[gord[a]]) { int t = gord[a]; gord[a] = gord[c]; gord[c] = t; }
            for (int r = 0; r < G; ++r) {
                const int g = gord[r];
                int32_t tl = c1[gi * 4 + g];
                if (tl < 0) continue;
                // A tile whose screened maximum t obeys t + c_i + E < (|y_i|^2 - D - slack) / 2
                // holds only rows with distance above D + slack: it cannot hold the minimum.
                if (bj >= 0 && gv[g] + qv.y + screen_err(qv, best, dl) < 0.5f * (ny2 - best - slack(best, dl))) continue;
                for (int e = 0; e < NE; ++e) {
                    const int32_t r = T == 16 ? tl * 16 + 4 * g + e : tl * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
                    if (r >= Fc.n) continue;
                    const int32_t j = perm[Fc.off + r];                 // packed row -> point
                    if (!valid[Fc.off + j]) continue;
                    float x[FD];
                    load_row(F, Fc.off + j, x);
                    float d = d2_row(q, x);
                    if (d < best || (d == best && j < bj)) { best = d; bj = j; }
                }
            }
            float E = screen_err(qv, best, dl);
            bool cert = a2 == -INFINITY || (bj >= 0 && best + slack(best, dl) < ny2 - 2.0f * (a2 + qv.y + E));
            if (cert) {
                nn[gi] = bj;
                dist[gi] = best;
            } else {
                fb = true;
                int k = atomicAdd(&fb_cnt[b.frag], 1);
                fb_row[Fq.off + k] = i;
                thr[Fq.off + k] = bj >= 0 ? 0.5f * (ny2 - best - slack(best, dl)) - qv.y - E : -INFINITY;
                if (k >= lst_cap(Fq) || bj < 0) {               // no list slot: rescan in float32
                    int r = atomicAdd(full_cnt, 1);
                    full_row[r] = i;
                    full_frag[r] = b.frag;
                }
            }
        }
    }
    unsigned long long bal = __ballot(fb);
    if ((threadIdx.x & 63) == 0 && bal && ps && Fq.pair >= 0)
        atomicAdd(&ps[Fq.pair].n_fallback, (unsigned long long)__popcll(bal));
}

// Exact re-rank of the collected candidates of each uncertified row.
__global__ void __launch_bounds__(256) k_rerank_list(const Frag *frag, const Blk *blk, const float *F,
                                                     const int32_t *valid, const int32_t *fb_row,
                                                     const int32_t *fb_cnt, const float *thr, const int32_t *lst,
                                                     const int32_t *lst_cnt, const int32_t *perm, int32_t *nn,
                                                     float *dist, int32_t *full_row, int32_t *full_frag,
                                                     int32_t *full_cnt) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fq = frag[b.frag];
    if (Fq.partner < 0) return;
    const int slot = b.start + threadIdx.x;
    const int nq = min(fb_cnt[b.frag], lst_cap(Fq));
    if (slot >= nq) return;
    const int32_t i = fb_row[Fq.off + slot];
    if (!(thr[Fq.off + slot] > -INFINITY)) return;              // already on the float32 rescan list
    const Frag &Fc = frag[Fq.partner];
    const int64_t ls = lst_base(Fq, b.frag) + slot;
    const int cnt = lst_cnt[ls];
    if (cnt > LCAP || cnt == 0) {
        int r = atomicAdd(full_cnt, 1);
        full_row[r] = i;
        full_frag[r] = b.frag;
        return;
    }
    float q[FD];
    load_row(F, Fq.off + i, q);
    float best = INFINITY;
    int32_t bj = -1;
    for (int k = 0; k < cnt; ++k) {
        const int32_t r = lst[ls * LCAP + k];                  // packed row
        if (r >= Fc.n) continue;
        const int32_t j = perm[Fc.off + r];
        if (!valid[Fc.off + j]) continue;
        float x[FD];
        load_row(F, Fc.off + j, x);
        float d = d2_row(q, x);
        if (d < best || (d == best && j < bj)) { best = d; bj = j; }
    }
    nn[Fq.off + i] = bj;
    dist[Fq.off + i] = best;
}

// Exact float32 rescan of the listed rows (grid-stride over the list).
__global__ void __launch_bounds__(256) k_fallback(const Frag *frag, const float *F, const int32_t *valid,
                                                  const int32_t *rows, const int32_t *rfrag, const int32_t *count,
                                                  int32_t *nn, float *dist) {
    __shared__ float sv[256];
    __shared__ int32_t si[256];
    const int n = *count;
    for (int r = blockIdx.x; r < n; r += gridDim.x) {
        const Frag &Fq = frag[rfrag[r]];
        const Frag &Fc = frag[Fq.partner];
        const int32_t i = rows[r];
        float q[FD];
        load_row(F, Fq.off + i, q);
        float best = INFINITY;
        int32_t bj = -1;
        for (int j = threadIdx.x; j < Fc.n; j += 256) {
            if (!valid[Fc.off + j]) continue;
            float x[FD];
            load_row(F, Fc.off + j, x);
            float d = d2_row(q, x);
            if (d < best) { best = d; bj = j; }
        }
        sv[threadIdx.x] = best;
        si[threadIdx.x] = bj;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                float w2 = sv[threadIdx.x + o];
                int32_t j2 = si[threadIdx.x + o];
                float w1 = sv[threadIdx.x];
                int32_t j1 = si[threadIdx.x];
                if (w2 < w1 || (w2 == w1 && j2 >= 0 && (j1 < 0 || j2 < j1))) { sv[threadIdx.x] = w2; si[threadIdx.x] = j2; }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            nn[Fq.off + i] = si[0];
            dist[Fq.off + i] = sv[0];
        }
        __syncthreads();
    }
}

template <bool COLLECT, int T, int SW, int SQB, int CH, int PRUNE>
static void screen_launch(const GridBufs &g, const uint16_t *pk, const ScreenScratch &S, PairState *ps,
                          hipStream_t s) {
    const int32_t *perm = S.perm, *rinv = S.rinv;
    if constexpr (T == 16) {
        if constexpr (COLLECT && PRUNE != 0)
            hipLaunchKernelGGL((k_screen_prc<SW, SQB, CH>), dim3(xcd_grid(g.nblk256)), dim3(SW * 64), 0, s,
                               (const Frag *)g.frag, (const Blk *)g.blk256, g.nblk256, pk, (const uint16_t *)S.cpk,
                               (const float4 *)S.cst, rinv, (const int32_t *)S.fb_row2, (const int32_t *)S.fb_cnt,
                               (const float *)S.thr2, S.lst, S.lst_cnt);
        else if constexpr (COLLECT)
            hipLaunchKernelGGL((k_screen<true, SW, SQB, CH>), dim3(xcd_grid(g.nblk256)), dim3(SW * 64), 0, s,
                               (const Frag *)g.frag, (const Blk *)g.blk256, g.nblk256, pk, perm, rinv, nullptr, nullptr,
                               nullptr, (const int32_t *)S.fb_row2, (const int32_t *)S.fb_cnt, (const float *)S.thr2,
                               S.lst, S.lst_cnt, nullptr);
        else if constexpr (PRUNE != 0)
            hipLaunchKernelGGL((k_screen_pr<SW, SQB, CH>), dim3(xcd_grid(g.nblk256)), dim3(SW * 64), 0, s, (const Frag *)g.frag,
                               (const Blk *)g.blk256, g.nblk256, pk, (const uint16_t *)S.cpk, (const float4 *)S.cst,
                               perm, S.c1, S.v2, S.v1, ps, (const uint64_t *)S.key1);
        else
            hipLaunchKernelGGL((k_screen<false, SW, SQB, CH>), dim3(g.nblk256), dim3(SW * 64), 0, s,
                               (const Frag *)g.frag, (const Blk *)g.blk256, g.nblk256, pk, perm, rinv, S.c1, S.v2, S.v1,
                               nullptr, nullptr, nullptr, nullptr, nullptr, ps);
    } else {
        if (COLLECT)
            hipLaunchKernelGGL((k_screen32<true, SW, SQB, CH>), dim3(xcd_grid(g.nblk256)), dim3(SW * 64), 0, s,
                               (const Frag *)g.frag, (const Blk *)g.blk256, g.nblk256, pk, perm, rinv, nullptr, nullptr,
                               nullptr, (const int32_t *)S.fb_row2, (const int32_t *)S.fb_cnt, (const float *)S.thr2,
                               S.lst, S.lst_cnt, nullptr);
        else
            hipLaunchKernelGGL((k_screen32<false, SW, SQB, CH>), dim3(g.nblk256), dim3(SW * 64), 0, s,
                               (const Frag *)g.frag, (const Blk *)g.blk256, g.nblk256, pk, perm, rinv, S.c1, S.v2, S.v1,
                               nullptr, nullptr, nullptr, nullptr, nullptr, ps);
    }
}

template <bool COLLECT>
static hipError_t launch_screen_c(int shape, const GridBufs &g, const uint16_t *pk, const ScreenScratch &S,
                                  PairState *ps, hipStream_t s) {
#define LSR_SHAPE(v) screen_launch<COLLECT, SCREEN_SHAPES[v].t, SCREEN_SHAPES[v].sw, SCREEN_SHAPES[v].sqb, \
                                     SCREEN_SHAPES[v].ch, SCREEN_SHAPES[v].prune>(g, pk, S, ps, s)
    switch (shape) {
    case 0: LSR_SHAPE(0); break;
    case 1: LSR_SHAPE(1); break;
    case 2: LSR_SHAPE(2); break;
    case 3: LSR_SHAPE(3); break;
    case 4: LSR_SHAPE(4); break;
    case 5: LSR_SHAPE(5); break;
    case 6: LSR_SHAPE(6); break;
    case 7: LSR_SHAPE(7); break;
    default: return hipErrorInvalidValue;
    }
#undef LSR_SHAPE
    return hipGetLastError();
}

static hipError_t launch_screen(bool collect, int shape, const GridBufs &g, const uint16_t *pk,
                                const ScreenScratch &S, PairState *ps, hipStream_t s) {
    return collect ? launch_screen_c<true>(shape, g, pk, S, ps, s) : launch_screen_c<false>(shape, g, pk, S, ps, s);
}

int screen_shapes() { return N_SCREEN_SHAPES; }

hipError_t launch_match_bf16(const GridBufs &g, DescBufs &d, MatchBufs &m, PairState *ps, void *scratch, int shape,
                             hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    ScreenScratch S = carve(scratch, g, nullptr);
    hipError_t e;
    if ((e = fill<int32_t>(S.fb_cnt, 0, g.nfrag, s)) != hipSuccess) return e;
    if ((e = fill<int32_t>(S.full_cnt, 0, 1, s)) != hipSuccess) return e;
    if ((e = fill<int32_t>(S.lst_cnt, 0, lst_slots(g), s)) != hipSuccess) return e;
    int npair = (g.nfrag + 1) / 2;
    hipLaunchKernelGGL(k_desc_mean, dim3(npair), dim3(256), 0, s, (const Frag *)g.frag, g.nfrag, (const float *)d.F,
                       (const int32_t *)d.valid, S.mean);
    if (shape < 0 || shape >= N_SCREEN_SHAPES) return hipErrorInvalidValue;
    // descriptor-space row order: principal directions, Hilbert keys, one sort of (fragment, key)
    hipLaunchKernelGGL(k_pca, dim3(npair), dim3(256), 0, s, (const Frag *)g.frag, g.nfrag, (const float *)d.F,
                       (const int32_t *)d.valid, (const float *)S.mean, S.pca);
    hipLaunchKernelGGL(k_mkey, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const float *)d.F, (const int32_t *)d.valid, (const float *)S.mean, (const float *)S.pca,
                       S.key0, S.idx0);
    size_t sb = S.sort_bytes;
    if ((e = rocprim::radix_sort_pairs(S.sort_tmp, sb, S.key0, S.key1, S.idx0, (uint32_t *)S.perm, (size_t)g.ntot, 0,
                                       sort_end_bit(g.nfrag), s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_rinv, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)S.perm, S.rinv);
    hipLaunchKernelGGL(k_pack, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const float *)d.F, (const int32_t *)d.valid, S.mean, (const int32_t *)S.rinv, d.pk, S.yq);
    if (SCREEN_SHAPES[shape].prune)
        hipLaunchKernelGGL(k_chunk_stats, dim3(g.nblk256), dim3(128), 0, s, (const Frag *)g.frag,
                           (const Blk *)g.blk256, (const uint16_t *)d.pk, S.cpk, S.cst);
    tmark("pack", s);
    if ((e = launch_screen(false, shape, g, d.pk, S, ps, s)) != hipSuccess) return e;
    tmark("screen", s);
    if (SCREEN_SHAPES[shape].t == 16)
        hipLaunchKernelGGL(k_rerank<16>, dim3(xcd_grid(g.nblk256)), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                           (const float *)d.F, (const int32_t *)d.valid, (const float4 *)S.yq, (const float *)S.mean,
                           (const int32_t *)S.perm, (const int32_t *)S.c1,
                           (const float *)S.v2, (const float *)S.v1, m.nn, m.dist, S.fb_row, S.thr, S.fb_cnt, S.full_row, S.full_frag,
                           S.full_cnt, ps, g.nblk256);
    else
        hipLaunchKernelGGL(k_rerank<32>, dim3(xcd_grid(g.nblk256)), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                           (const float *)d.F, (const int32_t *)d.valid, (const float4 *)S.yq, (const float *)S.mean,
                           (const int32_t *)S.perm, (const int32_t *)S.c1,
                           (const float *)S.v2, (const float *)S.v1, m.nn, m.dist, S.fb_row, S.thr, S.fb_cnt, S.full_row, S.full_frag,
                           S.full_cnt, ps, g.nblk256);
    tmark("rerank", s);
    // the uncertified rows of each fragment in packed-row order
    if ((e = fill<int32_t>(S.lmark, 0, g.ntot, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fb_mark, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)S.fb_row, (const int32_t *)S.fb_cnt, (const int32_t *)S.rinv, S.lmark);
    if ((e = exclusive_scan_i32(S.lmark, S.lpos, g.ntot, S.stmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fb_order, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)S.fb_row, (const float *)S.thr, (const int32_t *)S.fb_cnt,
                       (const int32_t *)S.rinv, (const int32_t *)S.lpos, S.fb_row2, S.thr2);
    if ((e = launch_screen(true, shape, g, d.pk, S, ps, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rerank_list, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const float *)d.F, (const int32_t *)d.valid, (const int32_t *)S.fb_row2,
                       (const int32_t *)S.fb_cnt, (const float *)S.thr2, (const int32_t *)S.lst,
                       (const int32_t *)S.lst_cnt, (const int32_t *)S.perm, m.nn, m.dist, S.full_row, S.full_frag,
                       S.full_cnt);
    tmark("collect", s);
    unsigned grid = (unsigned)std::min<int64_t>(g.ntot, 2048);
    hipLaunchKernelGGL(k_fallback, dim3(grid), dim3(256), 0, s, (const Frag *)g.frag, (const float *)d.F,
                       (const int32_t *)d.valid, (const int32_t *)S.full_row, (const int32_t *)S.full_frag,
                       (const int32_t *)S.full_cnt, m.nn, m.dist);
    return hipGetLastError();
}

}  // namespace lsr
