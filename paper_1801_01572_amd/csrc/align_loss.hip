// Robust alignment energy and its hand-written adjoint (eq. 2 with the line
// process eliminated, Psi of eq. 4):
//   E = sum_c mu s_c / (mu + s_c),  s_c = |r_c|^2,  r_c = R p_c + t - q_c.
// dE/ds = (mu / (mu + s))^2 = l_c (the optimal line-process weight), so
//   dE/dp_c = 2 l_c R^T r_c,  dE/dq_c = -2 l_c r_c,
//   dE/dxi  = sum_c 2 l_c [ p'_c x r_c ; r_c ]   for T <- Exp(xi) T (eq. 5's G^T r).
// l_c is recomputed in the backward pass, never stored.  Per-problem sums are
// reduced per block and then over blocks in a fixed order (deterministic).
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
                                              double *partial, float *dpx, float *dpy, float *dpz, float *dqx,
                                              float *dqy, float *dqz) {
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
            atomicAdd(&dpx[i], (float)(l * gx));
            atomicAdd(&dpy[i], (float)(l * gy));
            atomicAdd(&dpz[i], (float)(l * gz));
            atomicAdd(&dqx[j], (float)(-l * rx));
            atomicAdd(&dqy[j], (float)(-l * ry));
            atomicAdd(&dqz[j], (float)(-l * rz));
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

hipError_t launch_align(bool bwd, const float *const P[3], int64_t nP, const float *const Q[3], int64_t nQ,
                        const int32_t *corr,
                        const void *dev_tab, int64_t nblocks, const int64_t *dev_pblk, int nprob, const double *T,
                        const double *mu, const double *dE, double *partial, double *out, float *const dP[3],
                        float *const dQ[3], hipStream_t s) {
    int nv = bwd ? 6 : 1;
    if (nblocks > 0) {
        if (bwd)
            hipLaunchKernelGGL(k_align<true>, dim3((unsigned)nblocks), dim3(AT), 0, s, P[0], P[1], P[2], Q[0], Q[1],
                               Q[2], nP, nQ, corr, (const ABlk *)dev_tab, T, mu, dE, partial, dP[0], dP[1], dP[2], dQ[0],
                               dQ[1], dQ[2]);
        else
            hipLaunchKernelGGL(k_align<false>, dim3((unsigned)nblocks), dim3(AT), 0, s, P[0], P[1], P[2], Q[0], Q[1],
                               Q[2], nP, nQ, corr, (const ABlk *)dev_tab, T, mu, dE, partial, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr);
    }
    hipLaunchKernelGGL(k_align_reduce, dim3((nprob * nv + 63) / 64), dim3(64), 0, s, (const double *)partial,
                       dev_pblk, nprob, nv, out);
    return hipGetLastError();
}

}  // namespace lsr
