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
// (1 .. b-1 and b+1 .. n-1) are solved by block LDL^T for the right-hand
// side and the six columns that couple them to b, then b's 6x6 Schur
// complement gives its step and back-substitution the rest: O(n) per
// iteration.  Accepted when l >= l_min at the returned poses.
//
// One wave per candidate.  Edge blocks are formed one edge per lane and
// summed into node blocks one node per lane (each node in edge order, so
// the sums do not depend on scheduling).  Along a chain every 6x6 (and 6x7)
// block operation is spread over the lanes, one element each, exchanging
// operands through LDS; each Schur-complemented diagonal block is inverted
// by Gauss-Jordan elimination without pivoting, whose pivots are those of
// a Cholesky factorisation (a pivot <= 1e-12 tr(H) marks the system
// singular).  The next node's blocks are loaded while the current one is
// eliminated.  State lives in device scratch, FP64 throughout.
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

// Per-candidate scratch (doubles) for n nodes.
constexpr int NY = 42;      // a node's right-hand sides: 6 rows x (six coupling columns, -g)
struct Ws {
    double *T;      // n x 16 poses
    double *K;      // n x 36 edge blocks w J^T Lambda J (odometry edges 0 .. n-2, then the loop)
    double *r;      // n x 6 edge gradients w J^T Lambda xi
    double *D;      // n x 36 diagonal blocks H(k, k), then the inverses of their Schur complements
    double *O;      // n x 36: O[k] = H(k, k + 1)
    double *Y;      // n x 42 right-hand sides, then eliminated, then solved
};
__host__ __device__ inline size_t ws_doubles(int n) { return (size_t)n * (16 + 36 + 6 + 36 + 36 + NY); }
__device__ inline Ws carve(double *base, int n) {
    Ws w;
    w.T = base; base += 16 * n;
    w.K = base; base += 36 * n;
    w.r = base; base += 6 * n;
    w.D = base; base += 36 * n;
    w.O = base; base += 36 * n;
    w.Y = base;
    return w;
}

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// butterfly reductions: every lane ends with the same value
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// LDS of one wave's solve: one slot per lane (lanes past a block's 36 or 42
// elements write slots nobody reads, so no lane branches)
struct Lds {
    double a[64], b[64], inv[64], o[64], z[64];
    double y[2][64], x[64], t[64], s[64];
};

// Inverse of the symmetric positive definite 6x6 block whose element
// (l / 6, l % 6) lane l < 36 holds in v: Gauss-Jordan elimination in place,
// no pivoting (the pivot of step p is the p-th diagonal entry of the Schur
// complement, a Cholesky pivot).  The inverse lands in L.inv[0 .. 36) and
// each lane's element in v.  False (on every lane) on a pivot <= thr.
__device__ bool gj6(double &v, double thr, Lds &L) {
    const int l = threadIdx.x, i = l < 36 ? l : 35, r = i / 6, c = i % 6;
    L.a[l] = v;
    wsync();
    double *src = L.a, *nxt = L.b;
    for (int p = 0; p < 6; ++p) {
        const double piv = src[7 * p];
        if (!(piv > thr)) return false;
        const double ip = 1.0 / piv;
        const double mrc = src[i], mrp = src[6 * r + p], mpc = src[6 * p + c];
        const double up = mpc * ip, left = -mrp * ip, rest = mrc - mrp * mpc * ip;
        const double nv = r == p ? (c == p ? ip : up) : (c == p ? left : rest);
        double *dst = p == 5 ? L.inv : nxt;
        dst[l] = nv;
        wsync();
        nxt = src;
        src = dst;
        v = nv;
    }
    return true;
}

// Block LDL^T solve of the chain of nodes [lo, hi] (diagonal blocks D, upper
// blocks O) for the right-hand sides Y, lane-parallel within the wave:
// forward elimination D_k -= O_{k-1}^T D_{k-1}^-1 O_{k-1}, Y_k -= O_{k-1}^T
// D_{k-1}^-1 Y_{k-1}, then Y_k = D_k^-1 (Y_k - O_k Y_{k+1}) backwards.  D
// ends holding the inverted Schur complements.  False on a pivot <= thr.
__device__ bool chain_solve(const Ws &w, int lo, int hi, double thr, Lds &L) {
    const int l = threadIdx.x;
    const bool m36 = l < 36, m42 = l < NY;
    const int i36 = m36 ? l : 35, i42 = m42 ? l : 41;
    const int r6 = i36 / 6, c6 = i36 % 6, ry = i42 / 7, cy = i42 % 7;
    double d = w.D[36 * lo + i36], y = w.Y[NY * lo + i42], o = 0;
    int p = 0;
    for (int k = lo; k <= hi; ++k) {
        double nd = 0, ny = 0, no = 0;
        if (k < hi) {
            nd = w.D[36 * (k + 1) + i36];
            ny = w.Y[NY * (k + 1) + i42];
            no = w.O[36 * k + i36];
        }
        if (k > lo) {
            L.o[l] = o;
            wsync();
            double z = 0;                          // Z = D_{k-1}^-1 O_{k-1}
            for (int q = 0; q < 6; ++q) z += L.inv[6 * r6 + q] * L.o[6 * q + c6];
            L.z[l] = z;
            wsync();
            double sd = 0, sy = 0;
            for (int q = 0; q < 6; ++q) {
                sd += L.z[6 * q + r6] * L.o[6 * q + c6];
                sy += L.z[6 * q + ry] * L.y[p][7 * q + cy];
            }
            d -= sd;
            y -= sy;
        }
        if (m42) w.Y[NY * k + l] = y;
        L.y[p ^ 1][l] = y;
        if (!gj6(d, thr, L)) return false;
        if (m36) w.D[36 * k + l] = d;
        p ^= 1;
        d = nd;
        y = ny;
        o = no;
    }
    __syncthreads();                               // the inverses, read by rows below
    double yv = w.Y[NY * hi + i42], orow[6], drow[6];
    for (int q = 0; q < 6; ++q) { orow[q] = 0; drow[q] = w.D[36 * hi + 6 * ry + q]; }
    for (int k = hi; k >= lo; --k) {
        double nyv = 0, norow[6], ndrow[6];
        for (int q = 0; q < 6; ++q) norow[q] = ndrow[q] = 0;
        if (k > lo) {
            nyv = w.Y[NY * (k - 1) + i42];
            for (int q = 0; q < 6; ++q) {
                norow[q] = w.O[36 * (k - 1) + 6 * ry + q];
                ndrow[q] = w.D[36 * (k - 1) + 6 * ry + q];
            }
        }
        if (k < hi) {
            double s = 0;
            for (int q = 0; q < 6; ++q) s += orow[q] * L.x[7 * q + cy];
            yv -= s;
        }
        L.t[l] = yv;
        wsync();
        double x = 0;
        for (int q = 0; q < 6; ++q) x += drow[q] * L.t[7 * q + cy];
        if (m42) w.Y[NY * k + l] = x;
        L.x[l] = x;
        wsync();
        yv = nyv;
        for (int q = 0; q < 6; ++q) { orow[q] = norow[q]; drow[q] = ndrow[q]; }
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

// Energy at the poses T (every lane gets it): odometry edges one per lane.
__device__ double energy(const LoopArgs &a, const double *T, const lsr_edge &L, const double *Ll, double mu,
                         double *f_loop) {
    double E = 0, xi[6];
    for (int s = threadIdx.x; s < a.n - 1; s += 64) {
        pg::residual(a.odo[s].T, T + 16 * a.odo[s].i, T + 16 * a.odo[s].j, xi, nullptr);
        E += a.lambda * pg::quad(a.L_odo + 36 * s, xi);
    }
    E = pg::wave_sum(E);
    pg::residual(L.T, T + 16 * L.i, T + 16 * L.j, xi, nullptr);
    const double f = pg::quad(Ll, xi);
    *f_loop = f;
    return E + (mu > 0 ? mu * f / (mu + f) : 0.0);
}

// H(k, b) for a node k != b: minus the loop's block at its other end u (node
// 0 being fixed has none), minus the odometry blocks of b's chain neighbours.
__device__ __forceinline__ double coupling(const pg::Ws &w, int n, int k, int b, int u, int q, int c) {
    double s = 0;
    if (k == u && u >= 1) s -= w.K[36 * (n - 1) + 6 * q + c];
    if (k == b - 1) s -= w.K[36 * (b - 1) + 6 * q + c];
    if (k == b + 1) s -= w.K[36 * b + 6 * c + q];
    return s;
}

__global__ void __launch_bounds__(64) k_loop_solve(LoopArgs a) {
    __shared__ pg::Lds S;
    const int c = blockIdx.x, l = threadIdx.x, n = a.n;
    const pg::Ws w = pg::carve(a.scratch + (size_t)c * pg::ws_doubles(n), n);
    const lsr_edge L = a.loops[c];
    const double *Ll = a.L_loop + 36 * c;
    for (int k = l; k < 16 * n; k += 64) w.T[k] = a.T_init[k];
    __syncthreads();
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
        const int b = max(L.i, L.j), u = min(L.i, L.j);
        const bool m36 = l < 36, m42 = l < pg::NY;
        const int r6 = l / 6, c6 = l % 6, ry = m42 ? l / 7 : 0, cy = m42 ? l % 7 : 0;
        int it;
        for (it = 0; it < a.max_iter; ++it) {
            // edge blocks, one edge per lane
            for (int e = l; e < n; e += 64) {
                const lsr_edge &E = e < n - 1 ? a.odo[e] : L;
                const double *Le = e < n - 1 ? a.L_odo + 36 * e : Ll;
                double xi[6], J[36];
                pg::residual(E.T, w.T + 16 * E.i, w.T + 16 * E.j, xi, J);
                double wt = a.lambda;
                if (e == n - 1) { const double q = r.mu / (r.mu + pg::quad(Le, xi)); wt = q * q; }
                pg::edge_block(Le, J, xi, wt, w.K + 36 * e, w.r + 6 * e);
            }
            __syncthreads();
            // node blocks, one node per lane, its edges in order
            double trp = 0;
            for (int k = 1 + l; k < n; k += 64) {
                double D[36], g[6];
                for (int q = 0; q < 36; ++q) D[q] = 0;
                for (int q = 0; q < 6; ++q) g[q] = 0;
                const int es[3] = {k - 1, k <= n - 2 ? k : -1, (L.i == k || L.j == k) ? n - 1 : -1};
                for (int t = 0; t < 3; ++t) {
                    const int e = es[t];
                    if (e < 0) continue;
                    const lsr_edge &E = e < n - 1 ? a.odo[e] : L;
                    const double *K = w.K + 36 * e, *rr = w.r + 6 * e;
                    for (int q = 0; q < 36; ++q) D[q] += K[q];
                    if (E.i == k) for (int q = 0; q < 6; ++q) g[q] += rr[q];
                    else for (int q = 0; q < 6; ++q) g[q] -= rr[q];
                }
                for (int q = 0; q < 36; ++q) w.D[36 * k + q] = D[q];
                for (int q = 0; q < 6; ++q) trp += D[7 * q];
                if (k <= n - 2)
                    for (int q = 0; q < 36; ++q) w.O[36 * k + q] = -w.K[36 * k + q];
                for (int q = 0; q < 6; ++q) {
                    for (int cc = 0; cc < 6; ++cc) w.Y[pg::NY * k + 7 * q + cc] = coupling(w, n, k, b, u, q, cc);
                    w.Y[pg::NY * k + 7 * q + 6] = -g[q];
                }
            }
            const double thr = 1e-12 * pg::wave_sum(trp);
            __syncthreads();
            bool ok = true;
            if (b - 1 >= 1) ok = pg::chain_solve(w, 1, b - 1, thr, S);
            if (ok && b + 1 <= n - 1) ok = pg::chain_solve(w, b + 1, n - 1, thr, S);
            if (!ok) { status = LSR_DEGENERATE; break; }
            __syncthreads();
            // b's Schur complement (lanes < 42: six columns and the right-hand side)
            double sv = 0;
            if (m42) sv = cy < 6 ? w.D[36 * b + 6 * ry + cy] : w.Y[pg::NY * b + 7 * ry + 6];
            const int ks[3] = {u >= 1 && u != b - 1 ? u : -1, b - 1 >= 1 ? b - 1 : -1, b + 1 <= n - 1 ? b + 1 : -1};
            for (int t = 0; t < 3; ++t) {
                const int k = ks[t];
                if (k < 0 || !m42) continue;
                double s = 0;
                for (int q = 0; q < 6; ++q) s += coupling(w, n, k, b, u, q, ry) * w.Y[pg::NY * k + 7 * q + cy];
                sv -= s;
            }
            S.s[l] = sv;
            pg::wsync();
            double v = m36 ? S.s[7 * r6 + c6] : 0.0;
            if (!pg::gj6(v, thr, S)) { status = LSR_DEGENERATE; break; }
            double xb[6];
            for (int i = 0; i < 6; ++i) {
                double s = 0;
                for (int q = 0; q < 6; ++q) s += S.inv[6 * i + q] * S.s[7 * q + 6];
                xb[i] = s;
            }
            // steps and retraction T_k <- [Rod(w) | v] T_k, one node per lane
            double dmax = 0;
            for (int k = 1 + l; k < n; k += 64) {
                double x[6];
                for (int q = 0; q < 6; ++q) {
                    if (k == b) { x[q] = xb[q]; }
                    else {
                        double s = w.Y[pg::NY * k + 7 * q + 6];
                        for (int m = 0; m < 6; ++m) s -= w.Y[pg::NY * k + 7 * q + m] * xb[m];
                        x[q] = s;
                    }
                    dmax = fmax(dmax, fabs(x[q]));
                }
                double R[3][3], E4[16];
                pg::rod(x, R);
                for (int r3 = 0; r3 < 3; ++r3) {
                    for (int c3 = 0; c3 < 3; ++c3) E4[4 * r3 + c3] = R[r3][c3];
                    E4[4 * r3 + 3] = x[3 + r3];
                }
                E4[12] = E4[13] = E4[14] = 0;
                E4[15] = 1;
                pg::mul4(E4, w.T + 16 * k, w.T + 16 * k);
            }
            dmax = pg::wave_max(dmax);
            __syncthreads();
            if (dmax < a.tol) { ++it; break; }
        }
        __syncthreads();
        r.iters = it;
        r.energy = energy(a, w.T, L, Ll, r.mu, &r.f_loop);
        const double q = r.mu / (r.mu + r.f_loop);
        r.l = q * q;
        if (status != LSR_DEGENERATE) status = r.l >= a.l_min ? LSR_ACCEPTED : LSR_REJECTED;
        r.status = status;
    }
    if (l == 0) a.res[c] = r;
    if (a.T_out)
        for (int k = l; k < 16 * n; k += 64) a.T_out[(size_t)c * 16 * n + k] = w.T[k];
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
    hipLaunchKernelGGL(k_loop_solve, dim3(n_loops), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace lsr
