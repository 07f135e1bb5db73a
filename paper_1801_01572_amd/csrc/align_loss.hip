// Robust alignment energy and its hand-written adjoint (eq. 2 with the line
// process eliminated, Psi of eq. 4):
//   E = sum_c mu s_c / (mu + s_c),  s_c = |r_c|^2,  r_c = R p_c + t - q_c.
// dE/ds = (mu / (mu + s))^2 = l_c (the optimal line-process weight), so
//   dE/dp_c = 2 l_c R^T r_c,  dE/dq_c = -2 l_c r_c,
//   dE/dxi  = sum_c 2 l_c [ p'_c x r_c ; r_c ]   for T <- Exp(xi) T (eq. 5's G^T r).
// l_c is recomputed in the backward pass, never stored.  Per-problem sums are
// reduced per block and then over blocks in a fixed order; a point shared by
// several correspondences gets the FP64 sum of their contributions in
// ascending correspondence order (a counting sort of the correspondences by
// point, each point's short list ordered, then summed by one thread): every
// output is independent of scheduling.
#include <algorithm>

#include "lsr_internal.h"

namespace lsr {

constexpr int AT = 256;

struct ABlk {
    int32_t prob;
    int32_t pad;
    int64_t first, last;       // correspondence range of the block
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool BWD>
__global__ void __launch_bounds__(AT) k_align(const float *px, const float *py, const float *pz, const float *qx,
                                              const float *qy, const float *qz, int64_t nP, int64_t nQ,
                                              const int32_t *corr, const ABlk *blk,
                                              const double *Tall, const double *muall, const double *dEall,
                                              double *partial, double *cp, double *cq, int32_t *cntP,
                                              int32_t *cntQ) {
    constexpr int NV = BWD ? 6 : 1;
    __shared__ double sh[AT / 64][NV];
    const ABlk b = blk[blockIdx.x];
    const double *T = Tall + 16 * b.prob;
    const double mu = muall[b.prob];
    const double dE = BWD ? dEall[b.prob] : 1.0;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    int64_t c = b.first + threadIdx.x;
    int32_t i = -1, j = -1;
    if (c < b.last) { i = corr[2 * c]; j = corr[2 * c + 1]; }
    if (i >= 0 && i < nP && j >= 0 && j < nQ) {        // out-of-range pairs contribute nothing
        double p0 = px[i], p1 = py[i], p2 = pz[i];
        double x = T[0] * p0 + T[1] * p1 + T[2] * p2 + T[3];
        double y = T[4] * p0 + T[5] * p1 + T[6] * p2 + T[7];
        double z = T[8] * p0 + T[9] * p1 + T[10] * p2 + T[11];
        double rx = x - (double)qx[j], ry = y - (double)qy[j], rz = z - (double)qz[j];
        double s = rx * rx + ry * ry + rz * rz;
        if (!BWD) {
            acc[0] = mu * s / (mu + s);
        } else {
            double l = mu / (mu + s);
            l = 2.0 * dE * l * l;
            // R^T r
            double gx = T[0] * rx + T[4] * ry + T[8] * rz;
            double gy = T[1] * rx + T[5] * ry + T[9] * rz;
            double gz = T[2] * rx + T[6] * ry + T[10] * rz;
            cp[3 * c] = l * gx; cp[3 * c + 1] = l * gy; cp[3 * c + 2] = l * gz;
            cq[3 * c] = -l * rx; cq[3 * c + 1] = -l * ry; cq[3 * c + 2] = -l * rz;
            atomicAdd(&cntP[i], 1);           // integer counts: order-independent
            atomicAdd(&cntQ[j], 1);
            acc[0] = l * (y * rz - z * ry);
            acc[1] = l * (z * rx - x * rz);
            acc[2] = l * (x * ry - y * rx);
            acc[3] = l * rx; acc[4] = l * ry; acc[5] = l * rz;
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double v = wsum(acc[k]);
        if ((threadIdx.x & 63) == 0) sh[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double v = 0;
        for (int u = 0; u < AT / 64; ++u) v += sh[u][threadIdx.x];
        partial[(int64_t)blockIdx.x * NV + threadIdx.x] = v;
    }
}

// Correspondence c into its point's list (slot order arbitrary, fixed below).
__global__ void k_seg_fill(const int32_t *corr, int64_t m, int64_t nP, int64_t nQ, const int32_t *offP,
                           const int32_t *offQ, int32_t *curP, int32_t *curQ, int32_t *listP, int32_t *listQ) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const int32_t i = corr[2 * c], j = corr[2 * c + 1];
    if (!(i >= 0 && i < nP && j >= 0 && j < nQ)) return;
    listP[offP[i] + atomicAdd(&curP[i], 1)] = (int32_t)c;
    listQ[offQ[j] + atomicAdd(&curQ[j], 1)] = (int32_t)c;
}

// Point k: its correspondences in ascending order, contributions summed in
// FP64, added to the caller's float gradient once.
__global__ void k_seg_sum(int64_t n, const int32_t *off, int32_t *list, const double *contrib, float *gx, float *gy,
                          float *gz) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t b = off[k], e = off[k + 1];
    if (b == e) return;
    for (int32_t u = b + 1; u < e; ++u) {          // insertion sort: lists are short (usually one)
        const int32_t v = list[u];
        int32_t w = u - 1;
        while (w >= b && list[w] > v) { list[w + 1] = list[w]; --w; }
        list[w + 1] = v;
    }
    double sx = 0, sy = 0, sz = 0;
    for (int32_t u = b; u < e; ++u) {
        const int64_t c = list[u];
        sx += contrib[3 * c]; sy += contrib[3 * c + 1]; sz += contrib[3 * c + 2];
    }
    gx[k] += (float)sx;
    gy[k] += (float)sy;
    gz[k] += (float)sz;
}

// Per problem: sum of its blocks' partials in block order.
__global__ void k_align_reduce(const double *partial, const int64_t *pblk, int nprob, int nv, double *out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nprob * nv) return;
    int p = k / nv, v = k - p * nv;
    double s = 0;
    for (int64_t b = pblk[p]; b < pblk[p + 1]; ++b) s += partial[b * nv + v];
    out[k] = s;
}

int64_t align_blocks(const int64_t *coff, int nprob, void *host_tab, int64_t *pblk) {
    ABlk *t = (ABlk *)host_tab;
    int64_t nb = 0;
    for (int k = 0; k < nprob; ++k) {
        pblk[k] = nb;
        for (int64_t f = coff[k]; f < coff[k + 1]; f += AT) {
            if (t) t[nb] = ABlk{k, 0, f, f + AT < coff[k + 1] ? f + AT : coff[k + 1]};
            ++nb;
        }
    }
    pblk[nprob] = nb;
    return nb;
}

size_t align_block_bytes() { return sizeof(ABlk); }

size_t align_seg_bytes(int64_t m, int64_t nP, int64_t nQ) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 2 * al(sizeof(double) * 3 * (size_t)m) + 2 * al(sizeof(int32_t) * (size_t)m) +
           3 * al(sizeof(int32_t) * (size_t)(nP + 1)) + 3 * al(sizeof(int32_t) * (size_t)(nQ + 1)) +
           al(sizeof(int32_t) * scan_tmp_elems(std::max(nP, nQ) + 1));
}

hipError_t launch_align(bool bwd, const float *const P[3], int64_t nP, const float *const Q[3], int64_t nQ,
                        const int32_t *corr, int64_t m,
                        const void *dev_tab, int64_t nblocks, const int64_t *dev_pblk, int nprob, const double *T,
                        const double *mu, const double *dE, double *partial, double *out, float *const dP[3],
                        float *const dQ[3], char *seg, hipStream_t s) {
    int nv = bwd ? 6 : 1;
    hipError_t e = hipSuccess;
    if (!bwd) {
        if (nblocks > 0)
            hipLaunchKernelGGL(k_align<false>, dim3((unsigned)nblocks), dim3(AT), 0, s, P[0], P[1], P[2], Q[0], Q[1],
                               Q[2], nP, nQ, corr, (const ABlk *)dev_tab, T, mu, dE, partial, nullptr, nullptr,
                               nullptr, nullptr);
    } else {
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        char *o = seg;
        double *cp = (double *)o; o += al(sizeof(double) * 3 * (size_t)m);
        double *cq = (double *)o; o += al(sizeof(double) * 3 * (size_t)m);
        int32_t *listP = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)m);
        int32_t *listQ = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)m);
        int32_t *cntP = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)(nP + 1));
        int32_t *offP = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)(nP + 1));
        int32_t *curP = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)(nP + 1));
        int32_t *cntQ = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)(nQ + 1));
        int32_t *offQ = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)(nQ + 1));
        int32_t *curQ = (int32_t *)o; o += al(sizeof(int32_t) * (size_t)(nQ + 1));
        int32_t *stmp = (int32_t *)o;
        if ((e = fill<int32_t>(cntP, 0, nP + 1, s)) != hipSuccess || (e = fill<int32_t>(curP, 0, nP + 1, s)) ||
            (e = fill<int32_t>(cntQ, 0, nQ + 1, s)) || (e = fill<int32_t>(curQ, 0, nQ + 1, s)))
            return e;
        if (nblocks > 0)
            hipLaunchKernelGGL(k_align<true>, dim3((unsigned)nblocks), dim3(AT), 0, s, P[0], P[1], P[2], Q[0], Q[1],
                               Q[2], nP, nQ, corr, (const ABlk *)dev_tab, T, mu, dE, partial, cp, cq, cntP, cntQ);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // offsets over nP + 1 entries (the last, a zero count, gives the total)
        if ((e = exclusive_scan_i32(cntP, offP, nP + 1, stmp, s)) != hipSuccess) return e;
        if ((e = exclusive_scan_i32(cntQ, offQ, nQ + 1, stmp, s)) != hipSuccess) return e;
        if (m > 0) {
            hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, corr, m, nP, nQ,
                               (const int32_t *)offP, (const int32_t *)offQ, curP, curQ, listP, listQ);
            if (nP > 0)
                hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)((nP + 255) / 256)), dim3(256), 0, s, nP,
                                   (const int32_t *)offP, listP, (const double *)cp, dP[0], dP[1], dP[2]);
            if (nQ > 0)
                hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)((nQ + 255) / 256)), dim3(256), 0, s, nQ,
                                   (const int32_t *)offQ, listQ, (const double *)cq, dQ[0], dQ[1], dQ[2]);
        }
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_align_reduce, dim3((nprob * nv + 63) / 64), dim3(64), 0, s, (const double *)partial,
                       dev_pblk, nprob, nv, out);
    return hipGetLastError();
}

// T_out = [Rod(w) | v] T per problem, xi = (w, v).
__device__ void rod3(const double *w, double R[3][3]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
    double a, b;
    if (th < 1e-4) { a = 1 - th2 / 6 + th2 * th2 / 120; b = 0.5 - th2 / 24 + th2 * th2 / 720; }
    else { a = sin(th) / th; b = (1 - cos(th)) / th2; }
    const double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R[i][j] = (i == j) + a * K[i][j] + b * (K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j]);
}

__global__ void k_retract(int n, const double *xi, const double *T, double *Tout) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double R[3][3], o[16];
    rod3(xi + 6 * k, R);
    const double *A = T + 16 * k;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 4; ++c) o[4 * r + c] = R[r][0] * A[c] + R[r][1] * A[4 + c] + R[r][2] * A[8 + c];
        o[4 * r + 3] += xi[6 * k + 3 + r];
    }
    o[12] = A[12]; o[13] = A[13]; o[14] = A[14]; o[15] = A[15];
    for (int q = 0; q < 16; ++q) Tout[16 * k + q] = o[q];
}

// Gradient with respect to xi of E([Rod(w) | v] T) from the left-perturbation
// gradient (g_a, g_b) at [Rod(w) | v] T: dE/dw = J_l(w)^T (g_a - v x g_b),
// dE/dv = g_b, J_l the left Jacobian of SO(3).
__global__ void k_retract_grad(int n, const double *xi, const double *gl, double *gx) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double *w = xi + 6 * k, *v = xi + 6 * k + 3, *ga = gl + 6 * k, *gb = gl + 6 * k + 3;
    const double h[3] = {ga[0] - (v[1] * gb[2] - v[2] * gb[1]), ga[1] - (v[2] * gb[0] - v[0] * gb[2]),
                         ga[2] - (v[0] * gb[1] - v[1] * gb[0])};
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
    double a, b;            // J_l = I + a [w]x + b [w]x^2
    if (th < 1e-4) { a = 0.5 - th2 / 24 + th2 * th2 / 720; b = 1.0 / 6 - th2 / 120 + th2 * th2 / 5040; }
    else { a = (1 - cos(th)) / th2; b = (th - sin(th)) / (th2 * th); }
    const double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    for (int c = 0; c < 3; ++c) {        // (J_l^T h)_c = sum_r J_l[r][c] h_r
        double sum = 0;
        for (int r = 0; r < 3; ++r) {
            const double K2 = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
            sum += ((r == c) + a * K[r][c] + b * K2) * h[r];
        }
        gx[6 * k + c] = sum;
        gx[6 * k + 3 + c] = gb[c];
    }
}

hipError_t launch_retract(int n, const double *xi, const double *T, double *Tout, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_retract, dim3((n + 63) / 64), dim3(64), 0, s, n, xi, T, Tout);
    return hipGetLastError();
}

hipError_t launch_retract_grad(int n, const double *xi, const double *gl, double *gx, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_retract_grad, dim3((n + 63) / 64), dim3(64), 0, s, n, xi, gl, gx);
    return hipGetLastError();
}

}  // namespace lsr
