// Robust pose by graduated non-convexity on the line-process energy of
// Sec. V restricted to one fragment pair:
//   E_mu(T, l) = sum_c l_c |R p_c + t - q_c|^2 + mu sum_c (sqrt(l_c) - 1)^2   (eqs. 2-4)
// For fixed T the optimal weight is l_c = (mu / (mu + s_c))^2.  Each
// iteration linearises with G_c = [ -[p'_c]x | I ] (eq. 5), p'_c = R p_c + t,
// accumulates the 6x6 normal equations H = sum l G^T G and g = sum l G^T r in
// FP64, solves H xi = -g by Cholesky and updates T <- [Rod(omega) | v] T.
// mu starts at the squared diagonal of the correspondences' bounding box and
// is divided by gnc_div every gnc_every iterations down to max_corr^2; then up
// to polish_iter iterations at max_corr^2 until |xi|_inf < 1e-12.
//
// One block per pair; 27 FP64 sums per iteration reduced with wavefront
// shuffles and a fixed-order combine, so results are deterministic.  The
// correspondence loop is latency bound (one block per CU): 1024 threads and
// an unrolled loop keep several loads in flight per thread.
#include "lsr_internal.h"

namespace lsr {

constexpr int GT = 1024;          // one block per pair: 16 wavefronts share each iteration's sums
constexpr int GW = GT / 64;
constexpr int NS = 19;            // distinct entries: 13 of the symmetric H + 6 of g

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct CorrSrc {                   // correspondence coordinates: float (batched) or double (stage call)
    const float *pf, *qf;
    const double *pd, *qd;
    __device__ __forceinline__ void get(int64_t c, double p[3], double q[3]) const {
        if (pf) {
            p[0] = pf[3 * c]; p[1] = pf[3 * c + 1]; p[2] = pf[3 * c + 2];
            q[0] = qf[3 * c]; q[1] = qf[3 * c + 1]; q[2] = qf[3 * c + 2];
        } else {
            p[0] = pd[3 * c]; p[1] = pd[3 * c + 1]; p[2] = pd[3 * c + 2];
            q[0] = qd[3 * c]; q[1] = qd[3 * c + 1]; q[2] = qd[3 * c + 2];
        }
    }
};

struct GncShared {
    double red[GW][NS];
    double R[9], t[3];
    double xi[6];
    int ok;
    double mu;
};

__device__ void rod(const double w[3], double D[9]) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2), A, B;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        double h, c;                                  // sin th = 2 h c, 1 - cos th = 2 h^2
        sincos(0.5 * th, &h, &c);
        A = 2.0 * h * c / th;
        B = 2.0 * h * h / th2;
    }
    // I + A [w]x + B [w]x^2, with [w]x^2 = w w^T - th2 I
    D[0] = 1.0 + B * (w[0] * w[0] - th2); D[1] = -A * w[2] + B * w[0] * w[1]; D[2] = A * w[1] + B * w[0] * w[2];
    D[3] = A * w[2] + B * w[1] * w[0]; D[4] = 1.0 + B * (w[1] * w[1] - th2); D[5] = -A * w[0] + B * w[1] * w[2];
    D[6] = -A * w[1] + B * w[2] * w[0]; D[7] = A * w[0] + B * w[2] * w[1]; D[8] = 1.0 + B * (w[2] * w[2] - th2);
}

// Block-wide sums of v[0..n) (fixed order: waves by shuffles, then waves in order).
template <int N>
__device__ void block_sums(double (&v)[N], GncShared &sh) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < N; ++k) sh.red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0;
        for (int u = 0; u < GW; ++u) s += sh.red[u][threadIdx.x];
        sh.red[0][threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = sh.red[0][k];
    __syncthreads();
}

// One Gauss-Newton step at fixed mu; thread 0 solves and updates the pose.
__device__ void gn_step(const CorrSrc &src, int64_t m, double mu, GncShared &sh) {
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    const double *R = sh.R, *t = sh.t;
#pragma unroll 4
    for (int64_t c = threadIdx.x; c < m; c += GT) {
        double p[3], q[3];
        src.get(c, p, q);
        double x = R[0] * p[0] + R[1] * p[1] + R[2] * p[2] + t[0];
        double y = R[3] * p[0] + R[4] * p[1] + R[5] * p[2] + t[1];
        double z = R[6] * p[0] + R[7] * p[1] + R[8] * p[2] + t[2];
        double rx = x - q[0], ry = y - q[1], rz = z - q[2];
        double s = rx * rx + ry * ry + rz * rz;
        double l = mu / (mu + s);
        l *= l;
        // G = [[0, z, -y, 1,0,0], [-z, 0, x, 0,1,0], [y, -x, 0, 0,0,1]]
        // G^T G (upper triangle, row-major over 6x6) and G^T r
        double xx = x * x, yy = y * y, zz = z * z;
        // the 19 distinct sums: H's six zero entries (rows 0-2 against the
        // other rotation columns of I, and the off-diagonal of the I block) and
        // its three equal diagonal entries sum l are not accumulated separately
        acc[0] += l * (yy + zz);  acc[1] += l * (-x * y);  acc[2] += l * (-x * z);
        acc[3] += l * (-z);       acc[4] += l * (y);
        acc[5] += l * (xx + zz);  acc[6] += l * (-y * z);  acc[7] += l * (z);
        acc[8] += l * (-x);
        acc[9] += l * (xx + yy);  acc[10] += l * (-y);     acc[11] += l * (x);
        acc[12] += l;
        // G^T r = [p' x r ; r]
        acc[13] += l * (y * rz - z * ry);
        acc[14] += l * (z * rx - x * rz);
        acc[15] += l * (x * ry - y * rx);
        acc[16] += l * rx; acc[17] += l * ry; acc[18] += l * rz;
    }
    block_sums<NS>(acc, sh);
    if (threadIdx.x == 0) {
        // Fully unrolled (constant indices keep H and L in registers); the first
        // pivot at or below 1e-12 trace(H) marks the system degenerate.
        // upper triangle of H (row-major) from the distinct sums; -1: zero
        constexpr int HIDX[21] = {0, 1, 2, -1, 3, 4,      // row 0
                                  5, 6, 7, -1, 8,         // row 1
                                  9, 10, 11, -1,          // row 2
                                  12, -1, -1,             // row 3
                                  12, -1,                 // row 4
                                  12};                    // row 5
        double H[6][6];
        {
            int k = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int b = a; b < 6; ++b) {
                    const double h = HIDX[k] < 0 ? 0.0 : acc[HIDX[k] < 0 ? 0 : HIDX[k]];
                    H[a][b] = h; H[b][a] = h; ++k;
                }
        }
        double tr = H[0][0] + H[1][1] + H[2][2] + H[3][3] + H[4][4] + H[5][5];
        // one reciprocal square root per column (1 / L[j][j], hardware estimate and
        // two Newton steps: this block runs on one thread per iteration, so its
        // latency is the solve's), products elsewhere
        double L[6][6], il[6];
        bool okc = true;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double d = H[j][j];
#pragma unroll
            for (int u = 0; u < j; ++u) d -= L[j][u] * L[j][u];
            okc = okc && d > 1e-12 * tr;
            il[j] = rsqrt_nr(okc ? d : 1.0);
#pragma unroll
            for (int i = j + 1; i < 6; ++i) {
                double s = H[i][j];
#pragma unroll
                for (int u = 0; u < j; ++u) s -= L[i][u] * L[j][u];
                L[i][j] = s * il[j];
            }
        }
        const int ok = okc ? 1 : 0;
        sh.ok = ok;
        if (ok) {
            double yv[6], xi[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                double s = -acc[13 + i];
#pragma unroll
                for (int u = 0; u < i; ++u) s -= L[i][u] * yv[u];
                yv[i] = s * il[i];
            }
#pragma unroll
            for (int i = 5; i >= 0; --i) {
                double s = yv[i];
#pragma unroll
                for (int u = i + 1; u < 6; ++u) s -= L[u][i] * xi[u];
                xi[i] = s * il[i];
            }
            double D[9], Rn[9], tn[3];
            rod(xi, D);
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) Rn[3 * i + j] = D[3 * i] * R[j] + D[3 * i + 1] * R[3 + j] + D[3 * i + 2] * R[6 + j];
                tn[i] = D[3 * i] * t[0] + D[3 * i + 1] * t[1] + D[3 * i + 2] * t[2] + xi[3 + i];
            }
            for (int i = 0; i < 9; ++i) sh.R[i] = Rn[i];
            for (int i = 0; i < 3; ++i) sh.t[i] = tn[i];
            for (int i = 0; i < 6; ++i) sh.xi[i] = xi[i];
        }
    }
    __syncthreads();
}

__device__ void gnc_solve(const CorrSrc &src, int64_t m, double delta2, double div, int every, int max_iter,
                          int polish, GncShared &sh, PairState &out) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < 9; ++i) sh.R[i] = (i % 4 == 0) ? 1.0 : 0.0;
        sh.t[0] = sh.t[1] = sh.t[2] = 0.0;
        sh.ok = 1;
    }
    __syncthreads();
    int status = LSR_ACCEPTED, it = 0;
    double mu = delta2;
    if (m < 3) {
        status = LSR_DEGENERATE;
    } else {
        // bounding box of p and q together -> mu0 = squared diagonal
        double bb[6] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
        for (int64_t c = threadIdx.x; c < m; c += GT) {
            double p[3], q[3];
            src.get(c, p, q);
            for (int a = 0; a < 3; ++a) {
                bb[a] = fmin(bb[a], fmin(p[a], q[a]));
                bb[3 + a] = fmin(bb[3 + a], -fmax(p[a], q[a]));
            }
        }
        // min-reduce (a reduction of minima is order independent)
        for (int k = 0; k < 6; ++k)
            for (int o = 32; o > 0; o >>= 1) bb[k] = fmin(bb[k], __shfl_xor(bb[k], o, 64));
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) for (int k = 0; k < 6; ++k) sh.red[w][k] = bb[k];
        __syncthreads();
        for (int k = 0; k < 6; ++k) { bb[k] = sh.red[0][k]; for (int u = 1; u < GW; ++u) bb[k] = fmin(bb[k], sh.red[u][k]); }
        __syncthreads();
        double ex = -bb[3] - bb[0], ey = -bb[4] - bb[1], ez = -bb[5] - bb[2];
        mu = ex * ex + ey * ey + ez * ez;
        int anneal = 0;
        while (mu > delta2 && anneal < max_iter) {
            gn_step(src, m, mu, sh);
            if (!sh.ok) { status = LSR_DEGENERATE; break; }
            ++anneal; ++it;
            if (anneal % every == 0) { mu /= div; if (mu < delta2) mu = delta2; }
        }
        if (status != LSR_DEGENERATE) {
            mu = delta2;
            for (int k = 0; k < polish; ++k) {
                gn_step(src, m, mu, sh);
                if (!sh.ok) { status = LSR_DEGENERATE; break; }
                ++it;
                double mx = 0;
                for (int a = 0; a < 6; ++a) mx = fmax(mx, fabs(sh.xi[a]));
                if (mx < 1e-12) break;
            }
        }
    }
    // energy at the final pose
    double e[1] = {0.0};
    for (int64_t c = threadIdx.x; c < m; c += GT) {
        double p[3], q[3];
        src.get(c, p, q);
        const double *R = sh.R, *t = sh.t;
        double rx = R[0] * p[0] + R[1] * p[1] + R[2] * p[2] + t[0] - q[0];
        double ry = R[3] * p[0] + R[4] * p[1] + R[5] * p[2] + t[1] - q[1];
        double rz = R[6] * p[0] + R[7] * p[1] + R[8] * p[2] + t[2] - q[2];
        double s = rx * rx + ry * ry + rz * rz;
        e[0] += mu * s / (mu + s);
    }
    block_sums<1>(e, sh);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 16; ++i) out.T[i] = 0.0;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) out.T[4 * i + j] = sh.R[3 * i + j];
            out.T[4 * i + 3] = sh.t[i];
        }
        out.T[15] = 1.0;
        out.energy = e[0];
        out.mu_final = mu;
        out.iters = it;
        out.status = status;
    }
}

__global__ void __launch_bounds__(GT) k_gnc(const float *kp, const float *kq, PairState *ps, double delta2, double div,
                                            int every, int max_iter, int polish) {
    __shared__ GncShared sh;
    PairState &P = ps[blockIdx.x];
    int64_t m = (int64_t)P.n_consistent;
    CorrSrc src{kp + 3 * P.k_off, kq + 3 * P.k_off, nullptr, nullptr};
    gnc_solve(src, m, delta2, div, every, max_iter, polish, sh, P);
}

__global__ void __launch_bounds__(GT) k_gnc_direct(const double *p, const double *q, int64_t m, PairState *ps,
                                                   double delta2, double div, int every, int max_iter, int polish) {
    __shared__ GncShared sh;
    CorrSrc src{nullptr, nullptr, p, q};
    gnc_solve(src, m, delta2, div, every, max_iter, polish, sh, ps[0]);
}

hipError_t launch_gnc(const GridBufs &g, const MatchBufs &m, PairState *ps, int npairs, const lsr_params &prm,
                      hipStream_t s) {
    (void)g;
    if (npairs <= 0) return hipSuccess;
    double d2 = (double)prm.max_corr * (double)prm.max_corr;
    hipLaunchKernelGGL(k_gnc, dim3(npairs), dim3(GT), 0, s, (const float *)m.kp, (const float *)m.kq, ps, d2,
                       prm.gnc_div, prm.gnc_every, prm.gnc_max_iter, prm.polish_iter);
    return hipGetLastError();
}

hipError_t launch_gnc_direct(const double *p, const double *q, int64_t m, const lsr_params &prm, PairState *ps,
                             hipStream_t s) {
    double d2 = (double)prm.max_corr * (double)prm.max_corr;
    hipLaunchKernelGGL(k_gnc_direct, dim3(1), dim3(GT), 0, s, p, q, m, ps, d2, prm.gnc_div, prm.gnc_every,
                       prm.gnc_max_iter, prm.polish_iter);
    return hipGetLastError();
}

}  // namespace lsr
