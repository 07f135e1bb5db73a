// Verification of the returned pose (Algorithm 1's hypothesis test on the
// final transform): p is an inlier when some q lies within delta of T p
// (optionally with normal agreement (R n_p) . n_q >= cos), found on Q's 3-D
// grid, with T p, R n_p and the dot product in one fixed fma order, so that the
// predicate is a function of the inputs alone; inlier ratio =
// inliers / N_P, fitness = RMS distance of inliers to their nearest q.  The
// pair is accepted when the solve succeeded, at least min_consistent
// correspondences survived the consistency filter and the ratio reaches
// min_inlier_ratio.
#include "lsr_internal.h"

namespace lsr {

constexpr double FIX_SCALE = 1099511627776.0;   // 2^40: inlier d^2 / delta^2 in fixed point

__device__ __forceinline__ double xform_row(const double *r, double x, double y, double z, double c) {
    return __fma_rn(r[2], z, __fma_rn(r[1], y, __fma_rn(r[0], x, c)));
}

__global__ void __launch_bounds__(256) k_verify(const Frag *frag, const Blk *blk, const int32_t *cstart,
                                                const int32_t *ccount, const float4 *sp, const double *nxa, const double *nya,
                                                const double *nza, PairState *ps, double delta2, int normal_check,
                                                double ncos) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    if ((b.frag & 1) || P.partner < 0) return;
    const Frag &Q = frag[P.partner];
    PairState &S = ps[P.pair];
    int i = b.start + threadIdx.x;
    bool inl = false;
    double best = INFINITY;
    if (i < P.n) {
        int64_t s = P.off + i;                      // sorted position in P
        const double *T = S.T;
        const float4 ps4 = sp[s];
        double px = ps4.x, py = ps4.y, pz = ps4.z;
        // T p and R n_p: each row c + r0 x, then + r1 y, then + r2 z, one fma per step
        double x = xform_row(T, px, py, pz, T[3]);
        double y = xform_row(T + 4, px, py, pz, T[7]);
        double z = xform_row(T + 8, px, py, pz, T[11]);
        double rnx = 0, rny = 0, rnz = 0;
        if (normal_check) {
            double a = nxa[s], bb = nya[s], c = nza[s];
            rnx = xform_row(T, a, bb, c, 0.0);
            rny = xform_row(T + 4, a, bb, c, 0.0);
            rnz = xform_row(T + 8, a, bb, c, 0.0);
        }
        // cells that can hold a point within delta: 3 per axis, or 2 (p's cell and the
        // neighbour on the side of p's half) when delta is at most half a cell
        const double c = (double)Q.cell;
        const double fx = (x - (double)Q.ox) / c, fy = (y - (double)Q.oy) / c, fz = (z - (double)Q.oz) / c;
        const int cx = (int)floor(fx), cy = (int)floor(fy), cz = (int)floor(fz);
        int lx = cx - 1, ly = cy - 1, lz = cz - 1, hx = cx + 1, hy = cy + 1, hz = cz + 1;
        if (sqrt(delta2) <= 0.499999 * c) {
            lx = fx - cx < 0.5 ? cx - 1 : cx; hx = lx + 1;
            ly = fy - cy < 0.5 ? cy - 1 : cy; hy = ly + 1;
            lz = fz - cz < 0.5 ? cz - 1 : cz; hz = lz + 1;
        }
        int x0 = max(lx, 0), x1 = min(hx, Q.gx - 1);
        if (x0 <= x1) {
            for (int zz = max(lz, 0); zz <= min(hz, Q.gz - 1); ++zz)
                for (int yy = max(ly, 0); yy <= min(hy, Q.gy - 1); ++yy) {
                    int64_t row = Q.cell_off + ((int64_t)zz * Q.gy + yy) * Q.gx;
                    int32_t kb = cstart[row + x0], ke = cstart[row + x1] + ccount[row + x1];
                    for (int32_t k = kb; k < ke; ++k) {
                        if (normal_check && __fma_rn(rnz, nza[k], __fma_rn(rny, nya[k], rnx * nxa[k])) < ncos) continue;
                        const float4 q = sp[k];
                        double d2 = pdist2(x, y, z, (double)q.x, (double)q.y, (double)q.z);
                        best = fmin(best, d2);
                    }
                }
        }
        inl = best <= delta2;
    }
    unsigned long long fx = inl ? (unsigned long long)(best / delta2 * FIX_SCALE) : 0ull;
    unsigned long long bal = __ballot(inl);
    for (int o = 32; o > 0; o >>= 1) fx += __shfl_xor(fx, o, 64);
    if ((threadIdx.x & 63) == 0 && bal) {
        atomicAdd(&S.n_inliers, (unsigned long long)__popcll(bal));
        atomicAdd(&S.sum_d2_fixed, fx);
    }
}

hipError_t launch_verify(const GridBufs &g, const DescBufs &d, PairState *ps, float delta, int normal_check,
                         float normal_cos, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    double d2 = (double)delta * (double)delta;
    hipLaunchKernelGGL(k_verify, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)g.cstart, (const int32_t *)g.ccount, (const float4 *)g.sp, (const double *)d.nx, (const double *)d.ny, (const double *)d.nz, ps, d2,
                       normal_check, (double)normal_cos);
    return hipGetLastError();
}

__global__ void k_finalize(const Frag *frag, PairState *ps, int npairs, double delta2, int64_t min_cons,
                           double min_ratio, lsr_result *out) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= npairs) return;
    const PairState &S = ps[b];
    lsr_result r;
    for (int i = 0; i < 16; ++i) r.T[i] = S.T[i];
    int64_t nP = frag[2 * b].n;
    r.energy = S.energy;
    r.mu_final = S.mu_final;
    r.n_inliers = (int64_t)S.n_inliers;
    r.inlier_ratio = nP > 0 ? (double)S.n_inliers / (double)nP : 0.0;
    r.fitness = S.n_inliers ? sqrt((double)S.sum_d2_fixed / FIX_SCALE * delta2 / (double)S.n_inliers) : 0.0;
    r.n_valid_P = (int64_t)S.n_valid[0];
    r.n_valid_Q = (int64_t)S.n_valid[1];
    r.n_recip = (int64_t)S.n_recip;
    r.n_consistent = (int64_t)S.n_consistent;
    r.n_fallback_rows = (int64_t)S.n_fallback;
    r.n_screen_chunks = (int64_t)S.scr_chunks;
    r.n_screen_chunks_swept = (int64_t)S.scr_swept;
    r.iters = S.iters;
    if (S.status == LSR_DEGENERATE) r.status = LSR_DEGENERATE;
    else r.status = (r.n_consistent >= min_cons && r.inlier_ratio >= min_ratio) ? LSR_ACCEPTED : LSR_REJECTED;
    out[b] = r;
}

hipError_t launch_finalize(const GridBufs &g, PairState *ps, int npairs, const lsr_params &prm, lsr_result *out,
                           hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    double d2 = (double)prm.max_corr * (double)prm.max_corr;
    hipLaunchKernelGGL(k_finalize, dim3((npairs + 63) / 64), dim3(64), 0, s, (const Frag *)g.frag, ps, npairs, d2,
                       (int64_t)prm.min_consistent, (double)prm.min_inlier_ratio, out);
    return hipGetLastError();
}

}  // namespace lsr
