// RANSAC consensus, the pose stage of Algorithm 1 (Section IV): hypotheses
// of four random P points paired through the one-directional descriptor
// neighbour cache, pre-rejected by the similar-polygon test, fitted by least
// squares, and tested on all of P through Q's 3-D grid (eq. 1); the best
// hypothesis by inlier count is returned when its inlier ratio reaches the
// threshold.
//
// Hypothesis t fills slots s = 0..3 in order: slot s takes the first of up to
// 64 draws i = ((r >> 32) * N_P) >> 32 whose P point has a descriptor
// neighbour in Q and differs from the earlier slots, r the n-th SplitMix64
// output for n = (t << 8) | (s << 6) | attempt (the consistency filter's
// generator and counter layout).  A slot without such a draw voids the
// hypothesis.  Survivors of the polygon test are appended in any order; every
// later decision is order-free, and ties of the final choice are broken by
// the hypothesis index.
//
// Fit: Horn's closed form (1987): the rotation is the unit quaternion of the
// largest eigenvalue of the 4x4 matrix built from the cross-covariance of the
// centred pairs (Jacobi rotations here); the fit is refused when the two
// largest eigenvalues lie within 1e-9 of the largest magnitude (collinear or
// coincident points: the rotation is not unique).
//
// Test: p is an inlier when some q lies within delta of T p (optionally with
// normal agreement (R n_p) . n_q >= cos), T p and R n_p in the verification's
// pinned fma order; per hypothesis the inlier count and the sum of the
// inliers' squared nearest distances (FP64, a fixed reduction order).
// Choice: most inliers, then the smaller sum, then the lower hypothesis index;
// accepted when inliers / N_P reaches min_inlier_ratio.  One block tests one
// hypothesis (the paper's thread block per hypothesis with a parallel
// reduction); a block stops early once its hypothesis can no longer reach
// the largest count any hypothesis has completed, which cannot change the
// choice (every hypothesis that ties or beats the winner runs to the end).
#include "lsr_internal.h"

namespace lsr {

constexpr int RT = 256;           // threads of the test and choice blocks

// ---------------------------------------------------------------- hypotheses

__global__ void __launch_bounds__(256) k_ransac_hyp(const Frag *frag, const uint2 *cwords, const float4 *cpack,
                                                    const PairState *ps, int64_t n_hyp, uint64_t seed, double t2,
                                                    RansacBufs R) {
    const Frag &P = frag[0];
    const uint32_t nP = (uint32_t)P.n;
    if (ps->c_cnt < 4) return;                   // fewer than 4 eligible points: no hypothesis fills
    const uint2 *words = cwords + word_off(P, 0);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); base < n_hyp; base += stride) {
        const int64_t t = base + lane;
        bool ok = t < n_hyp;
        uint32_t id[4] = {0, 0, 0, 0};
        int pos[4] = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (!ok) continue;
            uint64_t z = seed + ((((uint64_t)t << 8) | ((uint64_t)s << 6)) + 1ull) * GAMMA;
            bool found = false;
            for (int a = 0; a < 64 && !found; ++a, z += GAMMA) {
                const uint32_t i = (uint32_t)(((uint64_t)splitmix64_hi(z) * nP) >> 32);
                const uint2 w = words[i >> 5];
                bool take = (w.x >> (i & 31)) & 1u;
#pragma unroll
                for (int u = 0; u < s; ++u) take = take && id[u] != i;
                if (take) {
                    id[s] = i;
                    pos[s] = (int)(w.y + (uint32_t)__popc(w.x & ((1u << (i & 31)) - 1u)));
                    found = true;
                }
            }
            ok = found;
        }
        if (ok) {
            float4 a[4], b[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) { a[k] = cpack[2 * pos[k]]; b[k] = cpack[2 * pos[k] + 1]; }
#pragma unroll
            for (int k = 0; k < 4; ++k) ok = ok && edge_ok(a[k], b[k], a[(k + 1) & 3], b[(k + 1) & 3], t2);
        }
        const unsigned long long bal = __ballot(ok);
        if (bal) {
            const int lead = __ffsll((long long)bal) - 1;
            unsigned long long first = 0;
            if (lane == lead) first = atomicAdd(&R.ctr[0], (unsigned long long)__popcll(bal));
            first = __shfl(first, lead, 64);
            if (ok) {
                const int64_t h = (int64_t)first + __popcll(bal & ((1ull << lane) - 1ull));
                if (h < R.cap) {
                    R.pos[h] = make_int4(pos[0], pos[1], pos[2], pos[3]);
                    R.t[h] = t;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- fit

// Eigen-decomposition of a symmetric 4x4 matrix by cyclic Jacobi rotations:
// on return the diagonal of A holds the eigenvalues and column k of V the
// eigenvector of A[k][k].
__device__ void jacobi_sym4(double A[4][4], double V[4][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, scale = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            scale += fabs(A[i][i]);
#pragma unroll
            for (int j = i + 1; j < 4; ++j) off += A[i][j] * A[i][j];
        }
        if (off == 0.0 || sqrt(off) <= 1e-20 * scale) break;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = p + 1; q < 4; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                // rotation angle that zeroes A[p][q]: tan = sign(h) / (|h| + sqrt(h^2 + 1))
                const double h = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double tn = copysign(1.0, h) / (fabs(h) + sqrt(h * h + 1.0));
                const double c = 1.0 / sqrt(tn * tn + 1.0), sn = tn * c;
#pragma unroll
                for (int k = 0; k < 4; ++k) {           // A <- A J
                    const double x = A[k][p], y = A[k][q];
                    A[k][p] = c * x - sn * y;
                    A[k][q] = sn * x + c * y;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {           // A <- J^T A
                    const double x = A[p][k], y = A[q][k];
                    A[p][k] = c * x - sn * y;
                    A[q][k] = sn * x + c * y;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {           // V <- V J
                    const double x = V[k][p], y = V[k][q];
                    V[k][p] = c * x - sn * y;
                    V[k][q] = sn * x + c * y;
                }
            }
    }
}

// Least-squares [R | t] (rows of 4) with q ~ R p + t from four pairs;
// false when the rotation is not unique.
__device__ bool horn_fit4(const double p[4][3], const double q[4][3], double T[12]) {
    double pm[3], qm[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pm[a] = (p[0][a] + p[1][a] + p[2][a] + p[3][a]) / 4.0;
        qm[a] = (q[0][a] + q[1][a] + q[2][a] + q[3][a]) / 4.0;
    }
    double S[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += (p[k][a] - pm[a]) * (q[k][b] - qm[b]);
            S[a][b] = acc;
        }
    // Horn's symmetric matrix: its eigenvector of the largest eigenvalue is the
    // quaternion (w, x, y, z) that maximises sum q'_k . R p'_k
    double N[4][4] = {
        {S[0][0] + S[1][1] + S[2][2], S[1][2] - S[2][1], S[2][0] - S[0][2], S[0][1] - S[1][0]},
        {S[1][2] - S[2][1], S[0][0] - S[1][1] - S[2][2], S[0][1] + S[1][0], S[2][0] + S[0][2]},
        {S[2][0] - S[0][2], S[0][1] + S[1][0], S[1][1] - S[0][0] - S[2][2], S[1][2] + S[2][1]},
        {S[0][1] - S[1][0], S[2][0] + S[0][2], S[1][2] + S[2][1], S[2][2] - S[0][0] - S[1][1]}};
    double V[4][4];
    jacobi_sym4(N, V);
    int k1 = 0;
#pragma unroll
    for (int k = 1; k < 4; ++k) k1 = N[k][k] > N[k1][k1] ? k : k1;
    double second = -INFINITY, big = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k != k1) second = fmax(second, N[k][k]);
        big = fmax(big, fabs(N[k][k]));
    }
    if (!(N[k1][k1] - second > 1e-9 * big)) return false;
    double w = V[0][k1], x = V[1][k1], y = V[2][k1], z = V[3][k1];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    const double Rm[3][3] = {{w * w + x * x - y * y - z * z, 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                             {2.0 * (x * y + w * z), w * w - x * x + y * y - z * z, 2.0 * (y * z - w * x)},
                             {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), w * w - x * x - y * y + z * z}};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T[4 * a] = Rm[a][0];
        T[4 * a + 1] = Rm[a][1];
        T[4 * a + 2] = Rm[a][2];
        T[4 * a + 3] = qm[a] - (Rm[a][0] * pm[0] + Rm[a][1] * pm[1] + Rm[a][2] * pm[2]);
    }
    return true;
}

__global__ void __launch_bounds__(256) k_ransac_fit(const float4 *cpack, RansacBufs R) {
    const int64_t ns = min((int64_t)R.ctr[0], R.cap);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < ns; h += stride) {
        const int4 ps4 = R.pos[h];
        const int pk[4] = {ps4.x, ps4.y, ps4.z, ps4.w};
        double p[4][3], q[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 a = cpack[2 * pk[k]], b = cpack[2 * pk[k] + 1];
            p[k][0] = a.x; p[k][1] = a.y; p[k][2] = a.z;
            q[k][0] = a.w; q[k][1] = b.x; q[k][2] = b.y;
        }
        double T[12];
        const bool ok = horn_fit4(p, q, T);
#pragma unroll
        for (int k = 0; k < 12; ++k) R.T[12 * h + k] = ok ? T[k] : (k % 5 == 0 ? 1.0 : 0.0);
        R.cnt[h] = ok ? 0 : -1;
        R.ss[h] = 0.0;
        if (ok) atomicAdd(&R.ctr[1], 1ull);
    }
}

// ---------------------------------------------------------------- test

__device__ __forceinline__ double xrow(const double *r, double x, double y, double z, double c) {
    return __fma_rn(r[2], z, __fma_rn(r[1], y, __fma_rn(r[0], x, c)));
}

// Squared distance from T p to its nearest q (with the normal check when
// asked), INFINITY when none lies within delta.  Stencil as the verification:
// the 2 x 2 x 2 cells nearest T p when delta is at most half a cell, else 3^3.
__device__ __forceinline__ double nearest_d2(const Frag &Q, const int32_t *cstart, const int32_t *ccount,
                                             const float4 *sp, const double *nxa, const double *nya,
                                             const double *nza, const double *T, double px, double py, double pz,
                                             double nx, double ny, double nz, double delta2, bool half,
                                             int normal_check, double ncos) {
    const double x = xrow(T, px, py, pz, T[3]);
    const double y = xrow(T + 4, px, py, pz, T[7]);
    const double z = xrow(T + 8, px, py, pz, T[11]);
    double rnx = 0, rny = 0, rnz = 0;
    if (normal_check) {
        rnx = xrow(T, nx, ny, nz, 0.0);
        rny = xrow(T + 4, nx, ny, nz, 0.0);
        rnz = xrow(T + 8, nx, ny, nz, 0.0);
    }
    const double c = (double)Q.cell;
    const double fx = (x - (double)Q.ox) / c, fy = (y - (double)Q.oy) / c, fz = (z - (double)Q.oz) / c;
    if (!(fx > -2.0 && fy > -2.0 && fz > -2.0 && fx < Q.gx + 1.0 && fy < Q.gy + 1.0 && fz < Q.gz + 1.0))
        return INFINITY;                                  // no cell of Q within reach (also NaN)
    const int cx = (int)floor(fx), cy = (int)floor(fy), cz = (int)floor(fz);
    int lx = cx - 1, ly = cy - 1, lz = cz - 1, hx = cx + 1, hy = cy + 1, hz = cz + 1;
    if (half) {
        lx = fx - cx < 0.5 ? cx - 1 : cx; hx = lx + 1;
        ly = fy - cy < 0.5 ? cy - 1 : cy; hy = ly + 1;
        lz = fz - cz < 0.5 ? cz - 1 : cz; hz = lz + 1;
    }
    double best = INFINITY;
    const int x0 = max(lx, 0), x1 = min(hx, Q.gx - 1);
    if (x0 > x1) return INFINITY;
    for (int zz = max(lz, 0); zz <= min(hz, Q.gz - 1); ++zz)
        for (int yy = max(ly, 0); yy <= min(hy, Q.gy - 1); ++yy) {
            const int64_t row = Q.cell_off + ((int64_t)zz * Q.gy + yy) * Q.gx;
            const int32_t kb = cstart[row + x0], ke = cstart[row + x1] + ccount[row + x1];
            for (int32_t k = kb; k < ke; ++k) {
                if (normal_check && __fma_rn(rnz, nza[k], __fma_rn(rny, nya[k], rnx * nxa[k])) < ncos) continue;
                const float4 q = sp[k];
                best = fmin(best, pdist2(x, y, z, (double)q.x, (double)q.y, (double)q.z));
            }
        }
    return best <= delta2 ? best : INFINITY;
}

// Points are tested in slices of RT per step; every SLICE steps the block
// compares its count plus the points left with the best count completed so
// far (R.ctr[2]) and stops when it cannot reach it.
constexpr int SLICE = 8;

__global__ void __launch_bounds__(RT) k_ransac_test(const Frag *frag, const int32_t *cstart, const int32_t *ccount,
                                                    const float4 *sp, const double *nxa, const double *nya,
                                                    const double *nza, RansacBufs R, double delta2,
                                                    int normal_check, double ncos) {
    __shared__ int s_cnt[RT / 64];
    __shared__ double s_ss[RT / 64];
    __shared__ int s_stop;
    const Frag &P = frag[0];
    const Frag &Q = frag[1];
    const int64_t ns = min((int64_t)R.ctr[0], R.cap);
    const bool half = sqrt(delta2) <= 0.499999 * (double)Q.cell;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t h = blockIdx.x; h < ns; h += gridDim.x) {
        if (R.cnt[h] < 0) continue;                       // block-uniform: no unique fit
        double T[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) T[k] = R.T[12 * h + k];
        int cnt = 0;
        double ss = 0.0;
        for (int i0 = 0; i0 < P.n; i0 += RT * SLICE) {
            for (int k = 0; k < SLICE; ++k) {
                const int i = i0 + k * RT + threadIdx.x;
                if (i < P.n) {
                    const int64_t s = P.off + i;
                    const float4 p = sp[s];
                    double nx = 0, ny = 0, nz = 0;
                    if (normal_check) { nx = nxa[s]; ny = nya[s]; nz = nza[s]; }
                    const double d2 = nearest_d2(Q, cstart, ccount, sp, nxa, nya, nza, T, p.x, p.y, p.z, nx, ny,
                                                 nz, delta2, half, normal_check, ncos);
                    if (d2 <= delta2) { ++cnt; ss += d2; }
                }
            }
            const int done = min(P.n, i0 + RT * SLICE);
            if (done < P.n) {
                int c = cnt;
                for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
                if (lane == 0) s_cnt[w] = c;
                __syncthreads();
                if (threadIdx.x == 0) {
                    int tot = 0;
                    for (int k = 0; k < RT / 64; ++k) tot += s_cnt[k];
                    const int64_t best = (int64_t)__atomic_load_n(&R.ctr[2], __ATOMIC_RELAXED);
                    s_stop = (int64_t)tot + (P.n - done) < best;
                }
                __syncthreads();
                const bool stop = s_stop;
                __syncthreads();
                if (stop) { cnt = -1; break; }
            }
        }
        if (cnt < 0) {                                    // cannot be chosen: recorded as below every count
            if (threadIdx.x == 0) { R.cnt[h] = -2; R.ss[h] = 0.0; }
            continue;
        }
        for (int o = 32; o > 0; o >>= 1) {
            cnt += __shfl_xor(cnt, o, 64);
            ss += __shfl_xor(ss, o, 64);
        }
        if (lane == 0) { s_cnt[w] = cnt; s_ss[w] = ss; }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            double sum = 0.0;
            for (int k = 0; k < RT / 64; ++k) { tot += s_cnt[k]; sum += s_ss[k]; }
            R.cnt[h] = tot;
            R.ss[h] = sum;
            atomicMax(&R.ctr[2], (unsigned long long)tot);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- choice

__device__ __forceinline__ bool better(int c1, double s1, int64_t t1, int c2, double s2, int64_t t2) {
    if (c1 != c2) return c1 > c2;
    if (s1 != s2) return s1 < s2;
    return t1 < t2;
}

__global__ void __launch_bounds__(1024) k_ransac_best(const Frag *frag, const PairState *ps, RansacBufs R,
                                                      int64_t n_hyp, double min_ratio, lsr_ransac_result *out) {
    __shared__ int s_c[1024];
    __shared__ double s_s[1024];
    __shared__ int64_t s_t[1024], s_h[1024];
    const int64_t ns = min((int64_t)R.ctr[0], R.cap);
    int bc = -3;
    double bs = 0.0;
    int64_t bt = INT64_MAX, bh = -1;
    for (int64_t h = threadIdx.x; h < ns; h += blockDim.x) {
        const int c = R.cnt[h];
        if (c < 0) continue;
        const double s = R.ss[h];
        const int64_t t = R.t[h];
        if (bh < 0 || better(c, s, t, bc, bs, bt)) { bc = c; bs = s; bt = t; bh = h; }
    }
    s_c[threadIdx.x] = bc; s_s[threadIdx.x] = bs; s_t[threadIdx.x] = bt; s_h[threadIdx.x] = bh;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int j = threadIdx.x + o;
            if (s_h[j] >= 0 && (s_h[threadIdx.x] < 0 ||
                                better(s_c[j], s_s[j], s_t[j], s_c[threadIdx.x], s_s[threadIdx.x], s_t[threadIdx.x]))) {
                s_c[threadIdx.x] = s_c[j]; s_s[threadIdx.x] = s_s[j];
                s_t[threadIdx.x] = s_t[j]; s_h[threadIdx.x] = s_h[j];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const int64_t nP = frag[0].n;
    lsr_ransac_result r;
    const int64_t h = s_h[0];
    for (int k = 0; k < 16; ++k) r.T[k] = (k % 5 == 0) ? 1.0 : 0.0;
    r.n_hypotheses = n_hyp;
    r.n_survivors = ns;
    r.n_fitted = (int64_t)R.ctr[1];
    r.n_valid_P = (int64_t)ps->n_valid[0];
    r.n_valid_Q = (int64_t)ps->n_valid[1];
    r.pad = 0;
    if (h < 0) {
        r.best = -1;
        r.n_inliers = 0;
        r.inlier_ratio = r.fitness = r.sum_d2 = 0.0;
        r.status = LSR_DEGENERATE;
    } else {
        for (int k = 0; k < 12; ++k) r.T[k] = R.T[12 * h + k];
        r.best = s_t[0];
        r.n_inliers = s_c[0];
        r.sum_d2 = s_s[0];
        r.inlier_ratio = nP > 0 ? (double)s_c[0] / (double)nP : 0.0;
        r.fitness = s_c[0] > 0 ? sqrt(s_s[0] / (double)s_c[0]) : 0.0;
        r.status = r.inlier_ratio >= min_ratio ? LSR_ACCEPTED : LSR_REJECTED;
    }
    *out = r;
}

// Per-survivor record in the caller's arrays (P indices of the members from
// the packed list).
__global__ void __launch_bounds__(256) k_ransac_trace(const float4 *cpack, RansacBufs R, lsr_ransac_trace tr) {
    const int64_t ns = min(min((int64_t)R.ctr[0], R.cap), tr.capacity);
    for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < ns; h += (int64_t)gridDim.x * blockDim.x) {
        const int4 p = R.pos[h];
        const int pk[4] = {p.x, p.y, p.z, p.w};
        if (tr.hyp) tr.hyp[h] = R.t[h];
        if (tr.members)
            for (int k = 0; k < 4; ++k) tr.members[4 * h + k] = __float_as_int(cpack[2 * pk[k] + 1].z);
        if (tr.n_inliers) tr.n_inliers[h] = R.cnt[h];
        if (tr.sum_d2) tr.sum_d2[h] = R.ss[h];
        if (tr.T)
            for (int k = 0; k < 16; ++k) tr.T[16 * h + k] = k < 12 ? R.T[12 * h + k] : (k == 15 ? 1.0 : 0.0);
    }
}

size_t ransac_bytes(int64_t cap) {
    return (size_t)cap * (sizeof(int4) + sizeof(int32_t) + 12 * sizeof(double) + sizeof(int32_t) + sizeof(double)) +
           8 * 256;
}

RansacBufs ransac_carve(void *mem, int64_t cap) {
    RansacBufs R;
    char *b = (char *)mem;
    auto take = [&](size_t bytes) { char *p = b; b += (bytes + 255) & ~size_t(255); return p; };
    R.ctr = (unsigned long long *)take(4 * sizeof(unsigned long long));
    R.pos = (int4 *)take(sizeof(int4) * (size_t)cap);
    R.t = (int32_t *)take(sizeof(int32_t) * (size_t)cap);
    R.T = (double *)take(12 * sizeof(double) * (size_t)cap);
    R.cnt = (int32_t *)take(sizeof(int32_t) * (size_t)cap);
    R.ss = (double *)take(sizeof(double) * (size_t)cap);
    R.cap = cap;
    return R;
}

// One pair: P = fragment 0, Q = fragment 1 of g; m.nn holds P's descriptor
// neighbours; d holds the estimated normals (sorted order).
hipError_t launch_ransac(const GridBufs &g, const DescBufs &d, MatchBufs &m, PairState *ps, RansacBufs R,
                         int64_t n_hyp, const lsr_params &prm, int32_t *scan_tmp, lsr_ransac_result *out,
                         const lsr_ransac_trace *tr, hipStream_t s) {
    hipError_t e;
    if ((e = fill<unsigned long long>(R.ctr, 0ull, 4, s)) != hipSuccess) return e;
    if ((e = launch_corr_pack(g, m, ps, true, scan_tmp, s)) != hipSuccess) return e;
    const Frag *fr = (const Frag *)g.frag;
    const double t2 = (double)prm.tau * (double)prm.tau;
    if (n_hyp > 0) {
        const int64_t nb = std::min<int64_t>((n_hyp + 255) / 256, 8192);
        hipLaunchKernelGGL(k_ransac_hyp, dim3((unsigned)nb), dim3(256), 0, s, fr, (const uint2 *)m.cwords,
                           (const float4 *)m.cpack, (const PairState *)ps, n_hyp, prm.seed, t2, R);
        const int64_t nf = std::min<int64_t>((std::min(n_hyp, R.cap) + 255) / 256, 4096);
        hipLaunchKernelGGL(k_ransac_fit, dim3((unsigned)nf), dim3(256), 0, s, (const float4 *)m.cpack, R);
        const int64_t nt = std::min<int64_t>(std::min(n_hyp, R.cap), 16384);
        const double d2 = (double)prm.max_corr * (double)prm.max_corr;
        hipLaunchKernelGGL(k_ransac_test, dim3((unsigned)nt), dim3(RT), 0, s, fr, (const int32_t *)g.cstart,
                           (const int32_t *)g.ccount, (const float4 *)g.sp, (const double *)d.nx,
                           (const double *)d.ny, (const double *)d.nz, R, d2, prm.normal_check,
                           (double)prm.normal_cos);
    }
    hipLaunchKernelGGL(k_ransac_best, dim3(1), dim3(1024), 0, s, fr, (const PairState *)ps, R, n_hyp,
                       (double)prm.min_inlier_ratio, out);
    if (tr && tr->capacity > 0)
        hipLaunchKernelGGL(k_ransac_trace, dim3(256), dim3(256), 0, s, (const float4 *)m.cpack, R, *tr);
    return hipGetLastError();
}

}  // namespace lsr
