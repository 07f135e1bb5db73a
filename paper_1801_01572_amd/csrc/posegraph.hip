// Loop verification by a line-process pose graph (Sec. V, eqs. 2-5).
//
// Edge information.  An edge (i, j, A) joins fragments i and j with a
// measured transform A from i's frame into j's.  Its correspondence set K
// holds the points p of fragment i with a point of fragment j within eps of
// A p (the verification predicate: A p and the squared distance in one
// pinned fma order, FP64, on j's 3-D grid), and its information matrix is
// Lambda = sum_{p in K} G_p^T G_p, G_p = [-[p]x | I] (eq. 5), which depends
// on K only through the count, the first moments s = sum p and the second
// moments M = sum p p^T:  Lambda = [[tr(M) I - M, [s]x], [-[s]x, |K| I]].
// One launch covers every edge of a chain: each edge is a (P, Q) pair of the
// batch layout, every point of its P fragment is one thread, and blocks
// write their ten moment sums (wave shuffles, then the block's waves in
// order) for a second kernel that adds each edge's blocks in order: the
// result does not depend on scheduling.
//
// Pose graph.  Per loop candidate, poses T_s (fragment -> world) of a chain
// whose odometry edge s joins s and s + 1; residual of an edge
// D = A^-1 T_j^-1 T_i with xi = (rotation vector of R_D, t_D) and energy
// f = xi^T Lambda xi; objective lambda sum f_odometry + mu f_loop / (mu +
// f_loop) (the line process l = (mu / (mu + f_loop))^2 eliminated, eqs. 2
// and 4), mu = tau^2 |K_loop|, node 0 fixed.  Gauss-Newton with l
// re-evaluated at every iterate, exact Jacobians under left perturbations
// T <- [Rod(w) | v] T (that of T_j is minus that of T_i).  The normal
// equations are block tridiagonal (the chain) plus the loop's coupling of
// nodes a < b; node b is eliminated last: the two chains left without it
// (1 .. b-1 and b+1 .. n-1) are solved by block LDL^T (6x6 Cholesky per
// node) for the right-hand side and the six columns that couple them to b,
// then b's 6x6 Schur complement gives its step and back-substitution the
// rest: O(n) per iteration.  Accepted when l >= l_min at the returned poses.
// One thread per candidate (small independent problems, FP64, state in
// device scratch).
#include <math.h>

#include "lsr_internal.h"

namespace lsr {

// ------------------------------------------------------------------ edge information

__device__ __forceinline__ double xrow(const double *r, double x, double y, double z, double c) {
    return __fma_rn(r[2], z, __fma_rn(r[1], y, __fma_rn(r[0], x, c)));
}

constexpr int NMOM = 10;    // count, sum x y z, sum xx xy xz yy yz zz

__global__ void __launch_bounds__(256) k_edge_moments(const Frag *frag, const Blk *blk, const int32_t *cstart,
                                                      const int32_t *ccount, const float4 *sp, const double *A_all,
                                                      double eps2, double *partial) {
    const Blk b = blk[blockIdx.x];
    const Frag &P = frag[b.frag];
    double m[NMOM];
    for (int k = 0; k < NMOM; ++k) m[k] = 0.0;
    const int i = b.start + threadIdx.x;
    const bool mine = (b.frag & 1) == 0 && i < P.n;
    if (mine) {
        const Frag &Q = frag[P.partner];
        const double *A = A_all + 16 * P.pair;
        const float4 p4 = sp[P.off + i];
        const double px = p4.x, py = p4.y, pz = p4.z;
        const double x = xrow(A, px, py, pz, A[3]);
        const double y = xrow(A + 4, px, py, pz, A[7]);
        const double z = xrow(A + 8, px, py, pz, A[11]);
        const double c = (double)Q.cell;
        const int cx = (int)floor((x - (double)Q.ox) / c), cy = (int)floor((y - (double)Q.oy) / c),
                  cz = (int)floor((z - (double)Q.oz) / c);
        bool hit = false;
        const int x0 = max(cx - 1, 0), x1 = min(cx + 1, Q.gx - 1);
        if (x0 <= x1)
            for (int zz = max(cz - 1, 0); zz <= min(cz + 1, Q.gz - 1) && !hit; ++zz)
                for (int yy = max(cy - 1, 0); yy <= min(cy + 1, Q.gy - 1) && !hit; ++yy) {
                    const int64_t row = Q.cell_off + ((int64_t)zz * Q.gy + yy) * Q.gx;
                    const int32_t kb = cstart[row + x0], ke = cstart[row + x1] + ccount[row + x1];
                    for (int32_t k = kb; k < ke; ++k) {
                        const float4 q = sp[k];
                        if (pdist2(x, y, z, (double)q.x, (double)q.y, (double)q.z) <= eps2) { hit = true; break; }
                    }
                }
        if (hit) {
            m[0] = 1.0; m[1] = px; m[2] = py; m[3] = pz;
            m[4] = px * px; m[5] = px * py; m[6] = px * pz; m[7] = py * py; m[8] = py * pz; m[9] = pz * pz;
        }
    }
    // block sums in a fixed order: within each wave by shuffles, then the waves in order
    __shared__ double ws[4][NMOM];
    for (int k = 0; k < NMOM; ++k) {
        double v = m[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NMOM)
        partial[(int64_t)blockIdx.x * NMOM + threadIdx.x] =
            ((ws[0][threadIdx.x] + ws[1][threadIdx.x]) + ws[2][threadIdx.x]) + ws[3][threadIdx.x];
}

// Edge e: its P fragment's blocks summed in order; Lambda from the moments.
__global__ void k_edge_info(const Frag *frag, const double *partial, int n_edges, double *info, int64_t *count) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_edges) return;
    const Frag &P = frag[2 * e];
    const int nb = (P.n + 255) / 256;
    double m[NMOM];
    for (int k = 0; k < NMOM; ++k) m[k] = 0.0;
    for (int bk = 0; bk < nb; ++bk)
        for (int k = 0; k < NMOM; ++k) m[k] += partial[(int64_t)(P.blk256_first + bk) * NMOM + k];
    const double n = m[0], sx = m[1], sy = m[2], sz = m[3];
    const double xx = m[4], xy = m[5], xz = m[6], yy = m[7], yz = m[8], zz = m[9];
    const double tr = xx + yy + zz;
    double L[36] = {tr - xx, -xy, -xz, 0, -sz, sy,
                    -xy, tr - yy, -yz, sz, 0, -sx,
                    -xz, -yz, tr - zz, -sy, sx, 0,
                    0, sz, -sy, n, 0, 0,
                    -sz, 0, sx, 0, n, 0,
                    sy, -sx, 0, 0, 0, n};
    for (int k = 0; k < 36; ++k) info[36 * e + k] = L[k];
    count[e] = (int64_t)n;
}

hipError_t launch_edge_info(const GridBufs &g, const double *A, int n_edges, float eps, double *partial,
                            double *info, int64_t *count, hipStream_t s) {
    if (n_edges == 0) return hipSuccess;
    if (g.nblk256 > 0) {
        hipLaunchKernelGGL(k_edge_moments, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag,
                           (const Blk *)g.blk256, (const int32_t *)g.cstart, (const int32_t *)g.ccount,
                           (const float4 *)g.sp, A, (double)eps * (double)eps, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_edge_info, dim3((n_edges + 63) / 64), dim3(64), 0, s, (const Frag *)g.frag,
                       (const double *)partial, n_edges, info, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pose graph

namespace pg {

// 4x4 row-major rigid transforms
__device__ void mul4(const double *A, const double *B, double *C) {
    double t[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            t[4 * r + c] = A[4 * r] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c] + A[4 * r + 3] * B[12 + c];
    for (int k = 0; k < 16; ++k) C[k] = t[k];
}
__device__ void inv4(const double *A, double *B) {
    double t[16];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) t[4 * r + c] = A[4 * c + r];
        t[4 * r + 3] = -(A[r] * A[3] + A[4 + r] * A[7] + A[8 + r] * A[11]);
    }
    t[12] = t[13] = t[14] = 0;
    t[15] = 1;
    for (int k = 0; k < 16; ++k) B[k] = t[k];
}

__device__ void skew(const double *v, double S[3][3]) {
    S[0][0] = 0; S[0][1] = -v[2]; S[0][2] = v[1];
    S[1][0] = v[2]; S[1][1] = 0; S[1][2] = -v[0];
    S[2][0] = -v[1]; S[2][1] = v[0]; S[2][2] = 0;
}

// rotation vector of R (angle in [0, pi])
__device__ void so3_log(const double R[3][3], double phi[3]) {
    double c = 0.5 * (R[0][0] + R[1][1] + R[2][2] - 1.0);
    const double v[3] = {0.5 * (R[2][1] - R[1][2]), 0.5 * (R[0][2] - R[2][0]), 0.5 * (R[1][0] - R[0][1])};
    const double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    c = fmin(1.0, fmax(-1.0, c));
    const double th = atan2(s, c);
    if (c > -0.99) {
        const double f = s > 1e-300 ? th / s : 1.0;
        for (int k = 0; k < 3; ++k) phi[k] = f * v[k];
        return;
    }
    double B[3][3];                    // (R + R^T) / 2 - c I = (1 - c) a a^T
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = 0.5 * (R[i][j] + R[j][i]) - (i == j ? c : 0.0);
    int best = 0;
    for (int k = 1; k < 3; ++k)
        if (B[k][k] > B[best][best]) best = k;
    double a[3] = {B[0][best], B[1][best], B[2][best]};
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) phi[k] = th * sg * a[k] / na;
}

// inverse left Jacobian of SO(3)
__device__ void jl_inv(const double phi[3], double J[3][3]) {
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], th = sqrt(th2);
    const double b = th < 1e-4 ? 1.0 / 12 + th2 / 720 : 1.0 / th2 - (1 + cos(th)) / (2 * th * sin(th));
    double K[3][3];
    skew(phi, K);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double k2 = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
            J[i][j] = (i == j) - 0.5 * K[i][j] + b * k2;
        }
}

__device__ void rod(const double w[3], double R[3][3]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2], th = sqrt(th2);
    double a, b;
    if (th < 1e-4) { a = 1 - th2 / 6 + th2 * th2 / 120; b = 0.5 - th2 / 24 + th2 * th2 / 720; }
    else { a = sin(th) / th; b = (1 - cos(th)) / th2; }
    double K[3][3];
    skew(w, K);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double k2 = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
            R[i][j] = (i == j) + a * K[i][j] + b * k2;
        }
}

// residual xi of edge (A, T_i, T_j) and J (6x6 row-major) for a left perturbation of T_i
__device__ void residual(const double *A, const double *Ti, const double *Tj, double xi[6], double *J) {
    double TjA[16], B[16], D[16];
    mul4(Tj, A, TjA);
    inv4(TjA, B);
    mul4(B, Ti, D);
    double RD[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) RD[r][c] = D[4 * r + c];
    double phi[3];
    so3_log(RD, phi);
    for (int k = 0; k < 3; ++k) { xi[k] = phi[k]; xi[3 + k] = D[4 * k + 3]; }
    if (!J) return;
    double Jl[3][3], S[3][3];
    const double d[3] = {D[3] - B[3], D[7] - B[7], D[11] - B[11]};
    jl_inv(phi, Jl);
    skew(d, S);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double a = 0, b = 0;
            for (int k = 0; k < 3; ++k) { a += Jl[r][k] * B[4 * k + c]; b += S[r][k] * B[4 * k + c]; }
            J[6 * r + c] = a; J[6 * r + 3 + c] = 0;
            J[6 * (3 + r) + c] = -b; J[6 * (3 + r) + 3 + c] = B[4 * r + c];
        }
}

__device__ double quad(const double *L, const double *x) {
    double s = 0;
    for (int a = 0; a < 6; ++a) {
        double t = 0;
        for (int b = 0; b < 6; ++b) t += L[6 * a + b] * x[b];
        s += x[a] * t;
    }
    return s;
}

// K = w J^T L J, r = w J^T L xi
__device__ void edge_block(const double *L, const double *J, const double *xi, double w, double *K, double *r) {
    double LJ[36];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += L[6 * a + k] * J[6 * k + b];
            LJ[6 * a + b] = s;
        }
    double Lx[6];
    for (int k = 0; k < 6; ++k) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += L[6 * k + m] * xi[m];
        Lx[k] = s;
    }
    for (int a = 0; a < 6; ++a) {
        for (int b = 0; b < 6; ++b) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += J[6 * k + a] * LJ[6 * k + b];
            K[6 * a + b] = w * s;
        }
        double s = 0;
        for (int k = 0; k < 6; ++k) s += J[6 * k + a] * Lx[k];
        r[a] = w * s;
    }
}

// Cholesky of a 6x6 SPD block in place (lower); false on a pivot <= thr
__device__ bool chol6(double *M, double thr) {
    for (int j = 0; j < 6; ++j) {
        double d = M[6 * j + j];
        for (int k = 0; k < j; ++k) d -= M[6 * j + k] * M[6 * j + k];
        if (!(d > thr)) return false;
        const double l = sqrt(d);
        M[6 * j + j] = l;
        for (int i = j + 1; i < 6; ++i) {
            double s = M[6 * i + j];
            for (int k = 0; k < j; ++k) s -= M[6 * i + k] * M[6 * j + k];
            M[6 * i + j] = s / l;
        }
    }
    return true;
}
// X (6 x nc, row-major, stride nc) <- M^-1 X with M = L L^T from chol6
__device__ void cholsolve6(const double *L, double *X, int nc) {
    for (int c = 0; c < nc; ++c) {
        double y[6];
        for (int i = 0; i < 6; ++i) {
            double s = X[nc * i + c];
            for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
            y[i] = s / L[6 * i + i];
        }
        for (int i = 5; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * X[nc * k + c];
            X[nc * i + c] = s / L[6 * i + i];
        }
    }
}

constexpr int NC = 7;       // right-hand sides of a chain solve: six coupling columns and the gradient

// Per-candidate scratch (doubles) for n nodes.
struct Ws {
    double *T;      // n x 16 poses
    double *Dg;     // n x 36 diagonal blocks (node 0 unused), then their factors
    double *Of;     // n x 36: Of[k] = H(k, k+1)
    double *g;      // n x 6
    double *Cb;     // n x 36: H(k, b) for the nodes coupled to b
    double *Y;      // n x 6 x NC right-hand sides / solutions
    double *x;      // n x 6 step
};
__host__ __device__ inline size_t ws_doubles(int n) { return (size_t)n * (16 + 36 + 36 + 6 + 36 + 6 * NC + 6); }
__device__ inline Ws carve(double *base, int n) {
    Ws w;
    w.T = base; base += 16 * n;
    w.Dg = base; base += 36 * n;
    w.Of = base; base += 36 * n;
    w.g = base; base += 6 * n;
    w.Cb = base; base += 36 * n;
    w.Y = base; base += 6 * NC * n;
    w.x = base;
    return w;
}

// Block LDL^T solve of the chain of nodes [lo, hi] (diagonal Dg, upper Of)
// for the NC right-hand sides in Y; factors Dg in place.  False on a pivot
// <= thr.
__device__ bool chain_solve(Ws &w, int lo, int hi, double thr) {
    for (int k = lo; k <= hi; ++k) {
        double *Dk = w.Dg + 36 * k;
        double *Yk = w.Y + 6 * NC * k;
        if (k > lo) {
            // W = O^T D_{k-1}^-1 with O = Of[k-1]: D_k -= W O, Y_k -= W Y_{k-1}
            const double *O = w.Of + 36 * (k - 1);
            const double *Lp = w.Dg + 36 * (k - 1);
            double Z[36];                       // Z = D_{k-1}^-1 O (6 x 6), so W = Z^T
            for (int i = 0; i < 36; ++i) Z[i] = O[i];
            cholsolve6(Lp, Z, 6);
            const double *Yp = w.Y + 6 * NC * (k - 1);
            for (int a = 0; a < 6; ++a) {
                for (int b = 0; b < 6; ++b) {
                    double s = 0;
                    for (int m = 0; m < 6; ++m) s += Z[6 * m + a] * O[6 * m + b];
                    Dk[6 * a + b] -= s;
                }
                for (int c = 0; c < NC; ++c) {
                    double s = 0;
                    for (int m = 0; m < 6; ++m) s += Z[6 * m + a] * Yp[NC * m + c];
                    Yk[NC * a + c] -= s;
                }
            }
        }
        if (!chol6(Dk, thr)) return false;
    }
    for (int k = hi; k >= lo; --k) {
        double *Yk = w.Y + 6 * NC * k;
        if (k < hi) {
            const double *O = w.Of + 36 * k;
            const double *Yn = w.Y + 6 * NC * (k + 1);
            for (int a = 0; a < 6; ++a)
                for (int c = 0; c < NC; ++c) {
                    double s = 0;
                    for (int m = 0; m < 6; ++m) s += O[6 * a + m] * Yn[NC * m + c];
                    Yk[NC * a + c] -= s;
                }
        }
        cholsolve6(w.Dg + 36 * k, Yk, NC);
    }
    return true;
}

}  // namespace pg

struct LoopArgs {
    int n;                        // nodes
    int n_loops;
    const double *T_init;         // n x 16
    const lsr_edge *odo;          // n - 1
    const double *L_odo;          // (n - 1) x 36
    const lsr_edge *loops;        // n_loops
    const double *L_loop;         // n_loops x 36
    const int64_t *cnt_loop;      // n_loops
    double lambda, tau2, l_min, tol;
    int max_iter;
    double *scratch;              // n_loops x ws_doubles(n)
    double *T_out;                // n_loops x n x 16, or NULL
    lsr_loop_result *res;
};

__device__ double energy(const LoopArgs &a, const double *T, const lsr_edge &L, const double *Ll, double mu,
                         double *f_loop) {
    double E = 0, xi[6];
    for (int s = 0; s < a.n - 1; ++s) {
        pg::residual(a.odo[s].T, T + 16 * a.odo[s].i, T + 16 * a.odo[s].j, xi, nullptr);
        E += a.lambda * pg::quad(a.L_odo + 36 * s, xi);
    }
    pg::residual(L.T, T + 16 * L.i, T + 16 * L.j, xi, nullptr);
    const double f = pg::quad(Ll, xi);
    *f_loop = f;
    return E + (mu > 0 ? mu * f / (mu + f) : 0.0);
}

__global__ void __launch_bounds__(64) k_loop_solve(LoopArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_loops) return;
    const int n = a.n;
    pg::Ws w = pg::carve(a.scratch + (size_t)c * pg::ws_doubles(n), n);
    const lsr_edge L = a.loops[c];
    const double *Ll = a.L_loop + 36 * c;
    for (int k = 0; k < 16 * n; ++k) w.T[k] = a.T_init[k];
    lsr_loop_result r;
    r.n_corr = a.cnt_loop[c];
    r.mu = a.tau2 * (double)r.n_corr;
    r.iters = 0;
    int status = LSR_ACCEPTED;
    if (r.n_corr <= 0) {
        r.energy = energy(a, w.T, L, Ll, 0.0, &r.f_loop);
        r.l = 0.0;
        r.status = LSR_REJECTED;
    } else {
        const int b = max(L.i, L.j);
        int it;
        for (it = 0; it < a.max_iter && n > 1; ++it) {
            for (int k = 0; k < 36 * n; ++k) { w.Dg[k] = 0; w.Of[k] = 0; w.Cb[k] = 0; }
            for (int k = 0; k < 6 * n; ++k) w.g[k] = 0;
            // every edge: K = w J^T L J, r = w J^T L xi into the blocks of its nodes
            for (int e = 0; e < n; ++e) {
                const lsr_edge &E = e < n - 1 ? a.odo[e] : L;
                const double *Le = e < n - 1 ? a.L_odo + 36 * e : Ll;
                double xi[6], J[36], K[36], rr[6];
                pg::residual(E.T, w.T + 16 * E.i, w.T + 16 * E.j, xi, J);
                double wt = a.lambda;
                if (e == n - 1) { const double q = r.mu / (r.mu + pg::quad(Le, xi)); wt = q * q; }
                pg::edge_block(Le, J, xi, wt, K, rr);
                const int i = E.i, j = E.j;
                for (int q = 0; q < 6; ++q) { w.g[6 * i + q] += rr[q]; w.g[6 * j + q] -= rr[q]; }
                for (int q = 0; q < 36; ++q) { w.Dg[36 * i + q] += K[q]; w.Dg[36 * j + q] += K[q]; }
                // off-diagonal H(i, j) = -K: chain neighbours go to Of, the loop's pair (a, b) to Cb[a]
                const int u = min(i, j), v = max(i, j);
                if (u == 0) continue;                       // node 0 is fixed
                if (v == b && e == n - 1) {
                    for (int q = 0; q < 36; ++q) w.Cb[36 * u + q] -= K[q];
                } else if (v == u + 1) {
                    for (int q = 0; q < 36; ++q) w.Of[36 * u + q] -= K[q];
                }
            }
            double tr = 0;
            for (int k = 1; k < n; ++k)
                for (int q = 0; q < 6; ++q) tr += w.Dg[36 * k + 7 * q];
            const double thr = 1e-12 * tr;
            // node b last: H(k, b) for k != b are Of[b-1] (k = b-1), Of[b]^T (k = b+1) and Cb[lo] (loop)
            if (b - 1 >= 1) for (int q = 0; q < 36; ++q) w.Cb[36 * (b - 1) + q] += w.Of[36 * (b - 1) + q];
            if (b + 1 <= n - 1)
                for (int r6 = 0; r6 < 6; ++r6)
                    for (int c6 = 0; c6 < 6; ++c6) w.Cb[36 * (b + 1) + 6 * r6 + c6] += w.Of[36 * b + 6 * c6 + r6];
            // right-hand sides of the two chains: six coupling columns and -g
            for (int k = 1; k < n; ++k) {
                if (k == b) continue;
                double *Yk = w.Y + 6 * pg::NC * k;
                for (int q = 0; q < 6; ++q) {
                    for (int c6 = 0; c6 < 6; ++c6) Yk[pg::NC * q + c6] = w.Cb[36 * k + 6 * q + c6];
                    Yk[pg::NC * q + 6] = -w.g[6 * k + q];
                }
            }
            bool ok = true;
            if (b - 1 >= 1) ok = pg::chain_solve(w, 1, b - 1, thr);
            if (ok && b + 1 <= n - 1) ok = pg::chain_solve(w, b + 1, n - 1, thr);
            if (!ok) { status = LSR_DEGENERATE; break; }
            // Schur complement on b: S = H_bb - sum_k H_kb^T Y_k, rhs -g_b - sum_k H_kb^T z_k
            double S[36], sb[6];
            for (int q = 0; q < 36; ++q) S[q] = w.Dg[36 * b + q];
            for (int q = 0; q < 6; ++q) sb[q] = -w.g[6 * b + q];
            for (int k = 1; k < n; ++k) {
                if (k == b) continue;
                const double *C = w.Cb + 36 * k;
                const double *Yk = w.Y + 6 * pg::NC * k;
                for (int r6 = 0; r6 < 6; ++r6) {
                    for (int c6 = 0; c6 < 6; ++c6) {
                        double s = 0;
                        for (int m = 0; m < 6; ++m) s += C[6 * m + r6] * Yk[pg::NC * m + c6];
                        S[6 * r6 + c6] -= s;
                    }
                    double s = 0;
                    for (int m = 0; m < 6; ++m) s += C[6 * m + r6] * Yk[pg::NC * m + 6];
                    sb[r6] -= s;
                }
            }
            if (!pg::chol6(S, thr)) { status = LSR_DEGENERATE; break; }
            pg::cholsolve6(S, sb, 1);
            double dmax = 0;
            for (int q = 0; q < 6; ++q) { w.x[6 * b + q] = sb[q]; dmax = fmax(dmax, fabs(sb[q])); }
            for (int k = 1; k < n; ++k) {
                if (k == b) continue;
                const double *Yk = w.Y + 6 * pg::NC * k;
                for (int q = 0; q < 6; ++q) {
                    double s = Yk[pg::NC * q + 6];
                    for (int m = 0; m < 6; ++m) s -= Yk[pg::NC * q + m] * sb[m];
                    w.x[6 * k + q] = s;
                    dmax = fmax(dmax, fabs(s));
                }
            }
            for (int k = 1; k < n; ++k) {                    // T_k <- [Rod(w) | v] T_k
                double R[3][3], E4[16];
                pg::rod(w.x + 6 * k, R);
                for (int r3 = 0; r3 < 3; ++r3) {
                    for (int c3 = 0; c3 < 3; ++c3) E4[4 * r3 + c3] = R[r3][c3];
                    E4[4 * r3 + 3] = w.x[6 * k + 3 + r3];
                }
                E4[12] = E4[13] = E4[14] = 0;
                E4[15] = 1;
                pg::mul4(E4, w.T + 16 * k, w.T + 16 * k);
            }
            if (dmax < a.tol) { ++it; break; }
        }
        r.iters = it;
        r.energy = energy(a, w.T, L, Ll, r.mu, &r.f_loop);
        const double q = r.mu / (r.mu + r.f_loop);
        r.l = q * q;
        if (status != LSR_DEGENERATE) status = r.l >= a.l_min ? LSR_ACCEPTED : LSR_REJECTED;
        r.status = status;
    }
    a.res[c] = r;
    if (a.T_out)
        for (int k = 0; k < 16 * n; ++k) a.T_out[(size_t)c * 16 * n + k] = w.T[k];
}

size_t loop_scratch_bytes(int n, int n_loops) { return sizeof(double) * pg::ws_doubles(n) * (size_t)n_loops; }

hipError_t launch_loop_solve(int n, const double *T_init, const lsr_edge *odo, const double *L_odo,
                             const lsr_edge *loops, int n_loops, const double *L_loop, const int64_t *cnt_loop,
                             const lsr_loop_params &prm, double *scratch, double *T_out, lsr_loop_result *res,
                             hipStream_t s) {
    if (n_loops == 0) return hipSuccess;
    LoopArgs a;
    a.n = n;
    a.n_loops = n_loops;
    a.T_init = T_init;
    a.odo = odo;
    a.L_odo = L_odo;
    a.loops = loops;
    a.L_loop = L_loop;
    a.cnt_loop = cnt_loop;
    a.lambda = prm.lambda;
    a.tau2 = prm.tau * prm.tau;
    a.l_min = prm.l_min;
    a.tol = prm.tol;
    a.max_iter = prm.max_iter;
    a.scratch = scratch;
    a.T_out = T_out;
    a.res = res;
    hipLaunchKernelGGL(k_loop_solve, dim3((n_loops + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace lsr
