/*
 * CPU FP64 oracle: loop verification by a line-process pose graph
 * (LoopSmart, Sec. V, eqs. 2-5).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Fragments s = 0..n-1 have poses T_s (fragment frame -> world, row-major
 * 4x4).  An edge (i, j, A) carries a measured transform A from fragment i's
 * frame into fragment j's (odometry s -> s+1, or a loop candidate from
 * registration; for consistent poses A = T_j^-1 T_i).  Its residual
 * transform is D = A^-1 T_j^-1 T_i (the paper's T_ij T_j^-1 T_i with
 * T_ij = A^-1), identity when the poses agree with the measurement, and its
 * 6-vector xi = (phi, t) holds the rotation vector of R_D and t_D.
 *
 * Edge energy (eq. 5): f = xi^T Lambda xi with Lambda = sum_{p in K} G_p^T G_p,
 * G_p = [-[p]x | I], p in fragment i's frame; K holds the points of P_i with a
 * point of P_j within eps of A p (the nearest neighbour within eps exists; G
 * depends on p only, so which neighbour does not matter).
 *
 * Objective (eq. 2 for one loop candidate, Psi of eq. 4):
 *   E(T, l) = lambda sum_s f_{s,s+1} + l f_loop + mu (sqrt(l) - 1)^2,
 * l in [0, 1].  Minimising over l gives l = (mu / (mu + f_loop))^2 and
 * E(T) = lambda sum_s f_s + mu f_loop / (mu + f_loop).
 * Readings: "mu = tau kappa" (kappa undefined) is read as
 * mu = tau^2 |K_loop|, so that l < 1/4 exactly when the loop's mean squared
 * point displacement at the optimum exceeds tau^2 (tau = 0.2 m, a distance
 * threshold); node 0 is held fixed (gauge); the solver (the paper uses g2o)
 * is Gauss-Newton with the line process re-evaluated at every iterate
 * (iteratively reweighted: weight lambda on odometry, l on the loop), exact
 * Jacobians of xi under left perturbations T <- [Rod(w) | v] T, a dense
 * Cholesky solve, stopping when |delta|_inf < tol or after max_iter steps.
 * A loop edge without correspondences is rejected without a solve (l = 0).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static void mat4_mul(const double *A, const double *B, double *C) {    /* C = A B (row-major 4x4) */
    double t[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0;
            for (int k = 0; k < 4; ++k) s += A[4 * r + k] * B[4 * k + c];
            t[4 * r + c] = s;
        }
    memcpy(C, t, sizeof t);
}

static void mat4_inv_rigid(const double *A, double *B) {              /* [R t]^-1 = [R^T, -R^T t] */
    double t[16] = {0};
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) t[4 * r + c] = A[4 * c + r];
        t[4 * r + 3] = -(A[r] * A[3] + A[4 + r] * A[7] + A[8 + r] * A[11]);
    }
    t[15] = 1;
    memcpy(B, t, sizeof t);
}

static void skew(const double v[3], double S[3][3]) {
    S[0][0] = 0; S[0][1] = -v[2]; S[0][2] = v[1];
    S[1][0] = v[2]; S[1][1] = 0; S[1][2] = -v[0];
    S[2][0] = -v[1]; S[2][1] = v[0]; S[2][2] = 0;
}

static void rod(const double w[3], double R[3][3]) {                    /* exp of a rotation vector */
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2), a, b;
    if (th < 1e-4) { a = 1 - th2 / 6 + th2 * th2 / 120; b = 0.5 - th2 / 24 + th2 * th2 / 720; }
    else { a = sin(th) / th; b = (1 - cos(th)) / th2; }
    double K[3][3];
    skew(w, K);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double k2 = 0;
            for (int k = 0; k < 3; ++k) k2 += K[i][k] * K[k][j];
            R[i][j] = (i == j) + a * K[i][j] + b * k2;
        }
}

/* rotation vector of R (the principal logarithm, angle in [0, pi]) */
static void so3_log(const double R[3][3], double phi[3]) {
    double c = 0.5 * (R[0][0] + R[1][1] + R[2][2] - 1.0);
    double v[3] = {0.5 * (R[2][1] - R[1][2]), 0.5 * (R[0][2] - R[2][0]), 0.5 * (R[1][0] - R[0][1])};
    double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (c > 1) c = 1;
    if (c < -1) c = -1;
    double th = atan2(s, c);
    if (c > -0.99) {                     /* v = sin(th) axis */
        double f = s > 1e-300 ? th / s : 1.0;
        for (int k = 0; k < 3; ++k) phi[k] = f * v[k];
        return;
    }
    /* near pi: (R + R^T)/2 - c I = (1 - c) a a^T */
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = 0.5 * (R[i][j] + R[j][i]) - (i == j ? c : 0.0);
    int best = 0;
    for (int k = 1; k < 3; ++k)
        if (B[k][k] > B[best][best]) best = k;
    double a[3] = {B[0][best], B[1][best], B[2][best]};
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int k = 0; k < 3; ++k) a[k] /= na;
    if (a[0] * v[0] + a[1] * v[1] + a[2] * v[2] < 0)
        for (int k = 0; k < 3; ++k) a[k] = -a[k];
    for (int k = 0; k < 3; ++k) phi[k] = th * a[k];
}

/* inverse left Jacobian of SO(3): Log(Exp(a) Exp(phi)) = phi + Jl^-1(phi) a + O(a^2) */
static void jl_inv(const double phi[3], double J[3][3]) {
    double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], th = sqrt(th2), b;
    if (th < 1e-4) b = 1.0 / 12 + th2 / 720;
    else b = 1.0 / th2 - (1 + cos(th)) / (2 * th * sin(th));
    double K[3][3];
    skew(phi, K);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double k2 = 0;
            for (int k = 0; k < 3; ++k) k2 += K[i][k] * K[k][j];
            J[i][j] = (i == j) - 0.5 * K[i][j] + b * k2;
        }
}

/* residual 6-vector of edge (A, T_i, T_j) and its Jacobian J with respect to
 * a left perturbation of T_i (that of T_j is -J) */
static void edge_residual(const double *A, const double *Ti, const double *Tj, double xi[6], double J[6][6]) {
    double TjA[16], B[16], D[16];
    mat4_mul(Tj, A, TjA);
    mat4_inv_rigid(TjA, B);                        /* B = A^-1 T_j^-1 */
    mat4_mul(B, Ti, D);                            /* D = B T_i */
    double RD[3][3], RB[3][3], tB[3] = {B[3], B[7], B[11]}, tD[3] = {D[3], D[7], D[11]};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) { RD[r][c] = D[4 * r + c]; RB[r][c] = B[4 * r + c]; }
    double phi[3];
    so3_log(RD, phi);
    for (int k = 0; k < 3; ++k) { xi[k] = phi[k]; xi[3 + k] = tD[k]; }
    if (!J) return;
    double Jl[3][3], S[3][3], d[3] = {tD[0] - tB[0], tD[1] - tB[1], tD[2] - tB[2]};
    jl_inv(phi, Jl);
    skew(d, S);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double a = 0, b = 0;
            for (int k = 0; k < 3; ++k) { a += Jl[r][k] * RB[k][c]; b += S[r][k] * RB[k][c]; }
            J[r][c] = a; J[r][3 + c] = 0;
            J[3 + r][c] = -b; J[3 + r][3 + c] = RB[r][c];
        }
}

static double quad(const double L[36], const double x[6]) {
    double s = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) s += x[a] * L[6 * a + b] * x[b];
    return s;
}

/* ------------------------------------------------------------ edge info */

void orc_edge_info(const float *ix, const float *iy, const float *iz, int64_t ni, const float *jx, const float *jy,
                   const float *jz, int64_t nj, const double *A, float eps, double *Lambda, int64_t *count) {
    uint8_t *fl = (uint8_t *)malloc((size_t)(ni > 0 ? ni : 1));
    orc_inliers(ix, iy, iz, ni, jx, jy, jz, nj, A, eps, fl);
    double L[36] = {0};
    int64_t m = 0;
    for (int64_t k = 0; k < ni; ++k) {
        if (!fl[k]) continue;
        double p[3] = {ix[k], iy[k], iz[k]};
        /* G = [-[p]x | I] (3 x 6) */
        double G[3][6] = {{0, p[2], -p[1], 1, 0, 0}, {-p[2], 0, p[0], 0, 1, 0}, {p[1], -p[0], 0, 0, 0, 1}};
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) L[6 * a + b] += G[0][a] * G[0][b] + G[1][a] * G[1][b] + G[2][a] * G[2][b];
        ++m;
    }
    memcpy(Lambda, L, sizeof L);
    *count = m;
    free(fl);
}

/* --------------------------------------------------------- pose graph */

static double total_energy(int32_t n, const double *T, const orc_edge *odo, const double *Lo, const orc_edge *loop,
                           const double *Ll, double lambda, double mu, double *f_loop) {
    double E = 0, xi[6];
    for (int32_t s = 0; s < n - 1; ++s) {
        edge_residual(odo[s].T, T + 16 * odo[s].i, T + 16 * odo[s].j, xi, NULL);
        E += lambda * quad(Lo + 36 * s, xi);
    }
    edge_residual(loop->T, T + 16 * loop->i, T + 16 * loop->j, xi, NULL);
    double f = quad(Ll, xi);
    *f_loop = f;
    return E + (mu > 0 ? mu * f / (mu + f) : 0.0);
}

int32_t orc_loop_solve(int32_t n, const double *T_init, const orc_edge *odo, const double *L_odo,
                       const orc_edge *loop, const double *L_loop, int64_t count_loop, const orc_loop_params *prm,
                       double *T_out, orc_loop_result *res) {
    memcpy(T_out, T_init, sizeof(double) * 16 * (size_t)n);
    memset(res, 0, sizeof *res);
    const double mu = prm->tau * prm->tau * (double)count_loop;
    res->mu = mu;
    if (count_loop <= 0) {
        res->l = 0;
        res->energy = total_energy(n, T_out, odo, L_odo, loop, L_loop, prm->lambda, 0.0, &res->f_loop);
        res->status = ORC_REJECTED;
        return res->status;
    }
    const int N = 6 * (n - 1);
    double *H = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N * N : 1));
    double *g = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *dx = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int status = ORC_ACCEPTED, it;
    for (it = 0; it < prm->max_iter && N > 0; ++it) {
        memset(H, 0, sizeof(double) * (size_t)N * N);
        memset(g, 0, sizeof(double) * (size_t)N);
        for (int32_t e = 0; e < n; ++e) {              /* n - 1 odometry edges, then the loop */
            const orc_edge *E = e < n - 1 ? odo + e : loop;
            const double *L = e < n - 1 ? L_odo + 36 * e : L_loop;
            double xi[6], J[6][6];
            edge_residual(E->T, T_out + 16 * E->i, T_out + 16 * E->j, xi, J);
            double w = prm->lambda;
            if (e == n - 1) { double f = quad(L, xi), r = mu / (mu + f); w = r * r; }
            double LJ[6][6], K[6][6], r6[6];
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) {
                    double s = 0;
                    for (int k = 0; k < 6; ++k) s += L[6 * a + k] * J[k][b];
                    LJ[a][b] = s;
                }
            for (int a = 0; a < 6; ++a) {
                for (int b = 0; b < 6; ++b) {
                    double s = 0;
                    for (int k = 0; k < 6; ++k) s += J[k][a] * LJ[k][b];
                    K[a][b] = w * s;
                }
                double s = 0;
                for (int k = 0; k < 6; ++k) {
                    double t = 0;
                    for (int m = 0; m < 6; ++m) t += L[6 * k + m] * xi[m];
                    s += J[k][a] * t;
                }
                r6[a] = w * s;
            }
            int bi = E->i - 1, bj = E->j - 1;          /* node 0 is fixed */
            for (int a = 0; a < 6; ++a) {
                if (bi >= 0) g[6 * bi + a] += r6[a];
                if (bj >= 0) g[6 * bj + a] -= r6[a];
                for (int b = 0; b < 6; ++b) {
                    if (bi >= 0) H[(size_t)(6 * bi + a) * N + 6 * bi + b] += K[a][b];
                    if (bj >= 0) H[(size_t)(6 * bj + a) * N + 6 * bj + b] += K[a][b];
                    if (bi >= 0 && bj >= 0) {
                        H[(size_t)(6 * bi + a) * N + 6 * bj + b] -= K[a][b];
                        H[(size_t)(6 * bj + a) * N + 6 * bi + b] -= K[b][a];
                    }
                }
            }
        }
        /* Cholesky H = L L^T in place (lower), then H dx = -g */
        double tr = 0;
        for (int a = 0; a < N; ++a) tr += H[(size_t)a * N + a];
        int ok = 1;
        for (int j = 0; j < N && ok; ++j) {
            double d = H[(size_t)j * N + j];
            for (int k = 0; k < j; ++k) d -= H[(size_t)j * N + k] * H[(size_t)j * N + k];
            if (!(d > 1e-12 * tr)) { ok = 0; break; }
            double Ljj = sqrt(d);
            H[(size_t)j * N + j] = Ljj;
            for (int i = j + 1; i < N; ++i) {
                double s = H[(size_t)i * N + j];
                for (int k = 0; k < j; ++k) s -= H[(size_t)i * N + k] * H[(size_t)j * N + k];
                H[(size_t)i * N + j] = s / Ljj;
            }
        }
        if (!ok) { status = ORC_DEGENERATE; break; }
        for (int i = 0; i < N; ++i) {
            double s = -g[i];
            for (int k = 0; k < i; ++k) s -= H[(size_t)i * N + k] * dx[k];
            dx[i] = s / H[(size_t)i * N + i];
        }
        for (int i = N - 1; i >= 0; --i) {
            double s = dx[i];
            for (int k = i + 1; k < N; ++k) s -= H[(size_t)k * N + i] * dx[k];
            dx[i] = s / H[(size_t)i * N + i];
        }
        double dmax = 0;
        for (int i = 0; i < N; ++i) if (fabs(dx[i]) > dmax) dmax = fabs(dx[i]);
        for (int32_t k = 1; k < n; ++k) {              /* T_k <- [Rod(w) | v] T_k */
            double R[3][3], E4[16] = {0};
            rod(dx + 6 * (k - 1), R);
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) E4[4 * r + c] = R[r][c];
                E4[4 * r + 3] = dx[6 * (k - 1) + 3 + r];
            }
            E4[15] = 1;
            mat4_mul(E4, T_out + 16 * k, T_out + 16 * k);
        }
        if (dmax < prm->tol) { ++it; break; }
    }
    res->iters = it;
    res->energy = total_energy(n, T_out, odo, L_odo, loop, L_loop, prm->lambda, mu, &res->f_loop);
    double r = mu / (mu + res->f_loop);
    res->l = r * r;
    if (status != ORC_DEGENERATE) status = res->l >= prm->l_min ? ORC_ACCEPTED : ORC_REJECTED;
    res->status = status;
    free(H); free(g); free(dx);
    return status;
}
