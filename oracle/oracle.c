/*
 * CPU FP64 oracle (test infrastructure only; see oracle.h).
 *
 * Each function follows the passage it cites, step by step, in double
 * precision, with no blocking or reordering beyond what the definition
 * states.  OpenMP only splits independent per-point or per-row work; every
 * per-point result is computed by one thread in a fixed order, so results do
 * not depend on the thread count.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NB 11          /* bins per feature (FPFH: 3 features x 11 bins) */
#define FD 33          /* descriptor length */

/* ------------------------------------------------------------------------ */
/* pinned squared distance between two float points                          */
/* ------------------------------------------------------------------------ */
static inline double dist2(double xi, double yi, double zi, double xj, double yj, double zj) {
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* ------------------------------------------------------------------------ */
/* O1: uniform grid over one cloud (Sec. IV, eq. 1, with floor, cell >= r)  */
/* The grid is only an index: neighbour sets are the exact radius sets and   */
/* are returned sorted by index, identical to the brute-force definition.    */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t key, idx; } kv_t;

typedef struct {
    double ox, oy, oz, cell;
    int64_t nx, ny, nz, n;
    kv_t *kv;                 /* sorted by (key, idx) */
} ogrid;

static int kv_cmp(const void *a, const void *b) {
    const kv_t *u = (const kv_t *)a, *v = (const kv_t *)b;
    if (u->key != v->key) return u->key < v->key ? -1 : 1;
    return (u->idx > v->idx) - (u->idx < v->idx);
}

static void grid_build(ogrid *g, const float *x, const float *y, const float *z, int64_t n, double r) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i) {
        double p[3] = {x[i], y[i], z[i]};
        for (int a = 0; a < 3; ++a) { if (p[a] < mn[a]) mn[a] = p[a]; if (p[a] > mx[a]) mx[a] = p[a]; }
    }
    if (n == 0) { mn[0] = mn[1] = mn[2] = 0; mx[0] = mx[1] = mx[2] = 0; }
    g->n = n;
    g->ox = mn[0]; g->oy = mn[1]; g->oz = mn[2];
    g->cell = r > 0 ? r * (1.0 + 1e-9) : 1.0;
    for (;;) {
        g->nx = (int64_t)floor((mx[0] - mn[0]) / g->cell) + 1;
        g->ny = (int64_t)floor((mx[1] - mn[1]) / g->cell) + 1;
        g->nz = (int64_t)floor((mx[2] - mn[2]) / g->cell) + 1;
        if ((double)g->nx * (double)g->ny * (double)g->nz < 4.0e18) break;
        g->cell *= 2.0;       /* keep keys in range; a larger cell is still exact */
    }
    g->kv = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix = (int64_t)floor(((double)x[i] - g->ox) / g->cell);
        int64_t iy = (int64_t)floor(((double)y[i] - g->oy) / g->cell);
        int64_t iz = (int64_t)floor(((double)z[i] - g->oz) / g->cell);
        g->kv[i].key = (iz * g->ny + iy) * g->nx + ix;
        g->kv[i].idx = i;
    }
    qsort(g->kv, (size_t)n, sizeof(kv_t), kv_cmp);
}

static void grid_free(ogrid *g) { free(g->kv); g->kv = NULL; }

static int64_t lower_key(const ogrid *g, int64_t key) {
    int64_t lo = 0, hi = g->n;
    while (lo < hi) { int64_t m = (lo + hi) / 2; if (g->kv[m].key < key) lo = m + 1; else hi = m; }
    return lo;
}

static int i64_cmp(const void *a, const void *b) {
    int64_t u = *(const int64_t *)a, v = *(const int64_t *)b;
    return (u > v) - (u < v);
}

/* All indices j with lo2 < d2(q, p_j) <= r2 (lo2 = 0 excludes coincident
 * points, lo2 = -1 includes them), sorted ascending.  Returns the count;
 * writes at most cap entries. */
static int64_t grid_query(const ogrid *g, const float *x, const float *y, const float *z,
                          double qx, double qy, double qz, double r2, double lo2,
                          int64_t *out, int64_t cap) {
    int64_t cx = (int64_t)floor((qx - g->ox) / g->cell);
    int64_t cy = (int64_t)floor((qy - g->oy) / g->cell);
    int64_t cz = (int64_t)floor((qz - g->oz) / g->cell);
    int64_t cnt = 0;
    for (int64_t dz = -1; dz <= 1; ++dz) {
        int64_t iz = cz + dz; if (iz < 0 || iz >= g->nz) continue;
        for (int64_t dy = -1; dy <= 1; ++dy) {
            int64_t iy = cy + dy; if (iy < 0 || iy >= g->ny) continue;
            for (int64_t dx = -1; dx <= 1; ++dx) {
                int64_t ix = cx + dx; if (ix < 0 || ix >= g->nx) continue;
                int64_t key = (iz * g->ny + iy) * g->nx + ix;
                for (int64_t s = lower_key(g, key); s < g->n && g->kv[s].key == key; ++s) {
                    int64_t j = g->kv[s].idx;
                    double d2 = dist2(qx, qy, qz, x[j], y[j], z[j]);
                    if (d2 > lo2 && d2 <= r2) { if (cnt < cap) out[cnt] = j; ++cnt; }
                }
            }
        }
    }
    if (cnt <= cap) qsort(out, (size_t)cnt, sizeof(int64_t), i64_cmp);
    return cnt;
}

/* CSR neighbourhoods of every point of one cloud (grid-backed). */
typedef struct { int64_t *off, *idx; } csr_t;

static csr_t csr_build(const float *x, const float *y, const float *z, int64_t n, double r) {
    csr_t c;
    ogrid g; grid_build(&g, x, y, z, n, r);
    double r2 = r * r;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel
    {
        int64_t cap = 4096; int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * cap);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int64_t k = grid_query(&g, x, y, z, x[i], y[i], z[i], r2, 0.0, tmp, cap);
            while (k > cap) { cap = 2 * k; tmp = (int64_t *)realloc(tmp, sizeof(int64_t) * cap);
                              k = grid_query(&g, x, y, z, x[i], y[i], z[i], r2, 0.0, tmp, cap); }
            cnt[i] = k;
        }
        free(tmp);
    }
    c.off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    c.off[0] = 0;
    for (int64_t i = 0; i < n; ++i) c.off[i + 1] = c.off[i] + cnt[i];
    c.idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(c.off[n] > 0 ? c.off[n] : 1));
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        grid_query(&g, x, y, z, x[i], y[i], z[i], r2, 0.0, c.idx + c.off[i], cnt[i]);
    free(cnt);
    grid_free(&g);
    return c;
}

static void csr_free(csr_t *c) { free(c->off); free(c->idx); }

int64_t orc_neighbors_grid(const float *x, const float *y, const float *z, int64_t n,
                           float r, int64_t *offsets, int64_t *idx, int64_t cap) {
    csr_t c = csr_build(x, y, z, n, (double)r);
    memcpy(offsets, c.off, sizeof(int64_t) * ((size_t)n + 1));
    int64_t tot = c.off[n];
    if (tot <= cap) memcpy(idx, c.idx, sizeof(int64_t) * (size_t)tot);
    csr_free(&c);
    return tot <= cap ? tot : -1;
}

int64_t orc_neighbors_brute(const float *x, const float *y, const float *z, int64_t n,
                            float r, int64_t *offsets, int64_t *idx, int64_t cap) {
    double r2 = (double)r * (double)r;
    int64_t tot = 0;
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double d2 = dist2(x[i], y[i], z[i], x[j], y[j], z[j]);
            if (d2 > 0.0 && d2 <= r2) { if (tot < cap) idx[tot] = j; ++tot; }
        }
        offsets[i + 1] = tot;
    }
    return tot <= cap ? tot : -1;
}

/* ------------------------------------------------------------------------ */
/* O0: voxel downsample (Algorithm 1, first step; leaf size in Sec. IV)     */
/* key = floor(coord / v) per axis; one output point per occupied voxel:     */
/* the mean position (rounded to float) and the normalised mean normal;      */
/* output ordered by ascending (kx, ky, kz).                                 */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t kx, ky, kz, idx; } vkey_t;

static int vkey_cmp(const void *a, const void *b) {
    const vkey_t *u = (const vkey_t *)a, *v = (const vkey_t *)b;
    if (u->kx != v->kx) return u->kx < v->kx ? -1 : 1;
    if (u->ky != v->ky) return u->ky < v->ky ? -1 : 1;
    if (u->kz != v->kz) return u->kz < v->kz ? -1 : 1;
    return (u->idx > v->idx) - (u->idx < v->idx);
}

int64_t orc_voxel(const float *x, const float *y, const float *z,
                  const float *nx, const float *ny, const float *nz, int64_t n, float v,
                  float *ox, float *oy, float *oz, float *onx, float *ony, float *onz) {
    double vd = (double)v;
    vkey_t *k = (vkey_t *)malloc(sizeof(vkey_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        k[i].kx = (int64_t)floor((double)x[i] / vd);
        k[i].ky = (int64_t)floor((double)y[i] / vd);
        k[i].kz = (int64_t)floor((double)z[i] / vd);
        k[i].idx = i;
    }
    qsort(k, (size_t)n, sizeof(vkey_t), vkey_cmp);
    int64_t m = 0;
    for (int64_t s = 0; s < n;) {
        int64_t e = s;
        double sx = 0, sy = 0, sz = 0, snx = 0, sny = 0, snz = 0;
        while (e < n && k[e].kx == k[s].kx && k[e].ky == k[s].ky && k[e].kz == k[s].kz) {
            int64_t i = k[e].idx;
            sx += x[i]; sy += y[i]; sz += z[i];
            snx += nx[i]; sny += ny[i]; snz += nz[i];
            ++e;
        }
        double c = (double)(e - s);
        ox[m] = (float)(sx / c); oy[m] = (float)(sy / c); oz[m] = (float)(sz / c);
        double nn = sqrt(snx * snx + sny * sny + snz * snz);
        if (nn > 0) { onx[m] = (float)(snx / nn); ony[m] = (float)(sny / nn); onz[m] = (float)(snz / nn); }
        else { int64_t i = k[s].idx; onx[m] = nx[i]; ony[m] = ny[i]; onz[m] = nz[i]; }
        ++m;
        s = e;
    }
    free(k);
    return m;
}

/* ------------------------------------------------------------------------ */
/* O2: normals by principal component analysis over N_rn(i) U {i}           */
/* (normal estimation radius, Sec. IV).  Symmetric 3x3 eigenproblem by      */
/* cyclic Jacobi rotations; the eigenvector of the smallest eigenvalue,      */
/* oriented to agree with the input normal.  Fewer than 3 points: the        */
/* normalised input normal.                                                  */
/* ------------------------------------------------------------------------ */
static void jacobi3(double A[3][3], double w[3], double V[3][3]) {
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) V[i][j] = (i == j);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double tr = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off == 0.0 || sqrt(off) <= 1e-18 * tr) break;
        for (int p = 0; p < 2; ++p) for (int q = p + 1; q < 3; ++q) {
            double apq = A[p][q];
            if (apq == 0.0) continue;
            double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
            double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            /* A <- J^T A J with J the (p,q) rotation */
            for (int k = 0; k < 3; ++k) {
                double akp = A[k][p], akq = A[k][q];
                A[k][p] = c * akp - s * akq;
                A[k][q] = s * akp + c * akq;
            }
            for (int k = 0; k < 3; ++k) {
                double apk = A[p][k], aqk = A[q][k];
                A[p][k] = c * apk - s * aqk;
                A[q][k] = s * apk + c * aqk;
            }
            for (int k = 0; k < 3; ++k) {
                double vkp = V[k][p], vkq = V[k][q];
                V[k][p] = c * vkp - s * vkq;
                V[k][q] = s * vkp + c * vkq;
            }
        }
    }
    for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

void orc_normals(const float *x, const float *y, const float *z,
                 const float *nx, const float *ny, const float *nz, int64_t n, float r_n,
                 double *nrm, double *gap, double *orient, int32_t *count) {
    csr_t nb = csr_build(x, y, z, n, (double)r_n);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = nb.off[i], e = nb.off[i + 1];
        int64_t m = e - b + 1;
        double nin[3] = {nx[i], ny[i], nz[i]};
        count[i] = (int32_t)(e - b);
        if (m < 3) {
            double l = sqrt(nin[0] * nin[0] + nin[1] * nin[1] + nin[2] * nin[2]);
            for (int a = 0; a < 3; ++a) nrm[3 * i + a] = l > 0 ? nin[a] / l : 0.0;
            gap[i] = -1.0; orient[i] = 1.0;
            continue;
        }
        /* the set N(i) U {i}, visited in ascending index order */
        double mu[3] = {0, 0, 0};
        int64_t s = b; int self_pending = 1;
        for (int64_t c = 0; c < m; ++c) {
            int64_t j;
            if (self_pending && (s == e || nb.idx[s] > i)) { j = i; self_pending = 0; }
            else j = nb.idx[s++];
            mu[0] += x[j]; mu[1] += y[j]; mu[2] += z[j];
        }
        for (int a = 0; a < 3; ++a) mu[a] /= (double)m;
        double C[3][3] = {{0}};
        s = b; self_pending = 1;
        for (int64_t c = 0; c < m; ++c) {
            int64_t j;
            if (self_pending && (s == e || nb.idx[s] > i)) { j = i; self_pending = 0; }
            else j = nb.idx[s++];
            double d[3] = {(double)x[j] - mu[0], (double)y[j] - mu[1], (double)z[j] - mu[2]};
            for (int a = 0; a < 3; ++a) for (int b2 = 0; b2 < 3; ++b2) C[a][b2] += d[a] * d[b2];
        }
        for (int a = 0; a < 3; ++a) for (int b2 = 0; b2 < 3; ++b2) C[a][b2] /= (double)m;
        double w[3], V[3][3];
        jacobi3(C, w, V);
        int o[3] = {0, 1, 2};
        for (int p = 0; p < 3; ++p) for (int q = p + 1; q < 3; ++q)
            if (w[o[q]] < w[o[p]]) { int t = o[p]; o[p] = o[q]; o[q] = t; }
        double v[3] = {V[0][o[0]], V[1][o[0]], V[2][o[0]]};
        double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int a = 0; a < 3; ++a) v[a] /= l;
        double dp = v[0] * nin[0] + v[1] * nin[1] + v[2] * nin[2];
        if (dp < 0) { for (int a = 0; a < 3; ++a) v[a] = -v[a]; dp = -dp; }
        for (int a = 0; a < 3; ++a) nrm[3 * i + a] = v[a];
        gap[i] = w[o[2]] > 0 ? (w[o[1]] - w[o[0]]) / w[o[2]] : 0.0;
        orient[i] = dp;
    }
    csr_free(&nb);
}

/* ------------------------------------------------------------------------ */
/* O3: simplified point feature histogram (FPFH definition, cited work).     */
/* For a pair (i, j): e = (p_j - p_i)/|p_j - p_i|; source s is the endpoint  */
/* whose normal makes the smaller angle with the line pointing to the other  */
/* endpoint (i on ties); u = n_s, v = u x e_st / |u x e_st|, w = u x v;      */
/* alpha = v.n_t, phi = u.e_st, theta = atan2(w.n_t, u.n_t).  11 bins per    */
/* feature over [-1,1], [-1,1], [-pi,pi]; each pair adds 1/k' per feature.   */
/* margin = distance (in bin units, or raw dot for the swap test) of the     */
/* closest decision to its boundary over all pairs of the point.            */
/* ------------------------------------------------------------------------ */
static inline int bin_of(double xbin) {           /* xbin = feature in bin units */
    double f = floor(xbin);
    if (f < 0) f = 0;
    if (f > NB - 1) f = NB - 1;
    return (int)f;
}

static inline double bin_margin(double xbin) {    /* distance to the nearest interior edge 1..10 */
    double r = floor(xbin + 0.5);
    if (r < 1) r = 1;
    if (r > NB - 1) r = NB - 1;
    return fabs(xbin - r);
}

/* theta lives on a circle: its bins also meet at the cut theta = +-pi
 * (bin units 0 and 11), where atan2 jumps from +pi to -pi. */
static inline double theta_margin(double xbin) {
    double r = floor(xbin + 0.5);
    if (r < 0) r = 0;
    if (r > NB) r = NB;
    return fabs(xbin - r);
}

/* Features of a pair seen from source u (normal n_s) towards the target
 * normal nt along es; returns 0 for a degenerate frame. */
static int features_from(const double *u, const double *nt, const double es[3], int bins[3], double *mb) {
    double v[3] = {u[1] * es[2] - u[2] * es[1], u[2] * es[0] - u[0] * es[2], u[0] * es[1] - u[1] * es[0]};
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (vn <= 1e-12) return 0;
    for (int a = 0; a < 3; ++a) v[a] /= vn;
    double w[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double alpha = v[0] * nt[0] + v[1] * nt[1] + v[2] * nt[2];
    double phi = u[0] * es[0] + u[1] * es[1] + u[2] * es[2];
    double theta = atan2(w[0] * nt[0] + w[1] * nt[1] + w[2] * nt[2], u[0] * nt[0] + u[1] * nt[1] + u[2] * nt[2]);
    double xa = NB * (alpha + 1.0) / 2.0;
    double xp = NB * (phi + 1.0) / 2.0;
    double xt = NB * (theta + M_PI) / (2.0 * M_PI);
    bins[0] = bin_of(xa); bins[1] = bin_of(xp); bins[2] = bin_of(xt);
    double m = bin_margin(xa);
    if (bin_margin(xp) < m) m = bin_margin(xp);
    if (theta_margin(xt) < m) m = theta_margin(xt);
    /* conditioning: v = u x e / |u x e| and theta = atan2(y, x) turn rounding
     * of order 1e-16 into errors of 1e-16 / vn and 1e-16 / |(x, y)|; below 1e-6
     * the bins are not decided by the inputs */
    double tx = u[0] * nt[0] + u[1] * nt[1] + u[2] * nt[2];
    double ty = w[0] * nt[0] + w[1] * nt[1] + w[2] * nt[2];
    double rt = sqrt(tx * tx + ty * ty);
    if (vn < 1e-6 && vn < m) m = vn;
    if (rt < 1e-6 && rt < m) m = rt;
    *mb = m;
    return 1;
}

/* Pair (i, j): returns 0 if the pair is skipped (degenerate frame).  The
 * margin is the smallest distance of a decision to its boundary; the source
 * test counts only when choosing the other source would change a bin. */
static int pair_features(const double pi[3], const double ni[3], const double pj[3], const double nj[3],
                         int bins[3], double *margin) {
    double dv[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
    double d = sqrt(fma(dv[2], dv[2], fma(dv[1], dv[1], dv[0] * dv[0])));
    double e[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
    double ne[3] = {-e[0], -e[1], -e[2]};
    double ci = ni[0] * e[0] + ni[1] * e[1] + ni[2] * e[2];
    double cj = nj[0] * e[0] + nj[1] * e[1] + nj[2] * e[2];
    int src_i = ci >= -cj;
    double mb;
    int ok = src_i ? features_from(ni, nj, e, bins, &mb) : features_from(nj, ni, ne, bins, &mb);
    double m = ok ? mb : INFINITY;
    double sw = fabs(ci + cj);
    if (sw < 1e-6) {                 /* source choice near its boundary: does it matter? */
        int b2[3]; double mb2;
        int ok2 = src_i ? features_from(nj, ni, ne, b2, &mb2) : features_from(ni, nj, e, b2, &mb2);
        int same = ok == ok2 && (!ok || (b2[0] == bins[0] && b2[1] == bins[1] && b2[2] == bins[2]));
        if (same) { if (ok2 && mb2 < m) m = mb2; }
        else if (sw < m) m = sw;
    }
    *margin = m;
    return ok;
}

static void spfh_core(const float *x, const float *y, const float *z, const double *nrm, int64_t n,
                      const csr_t *nb, double *spfh, int32_t *k, int32_t *kprime, double *margin) {
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t cnt[FD] = {0};
        int64_t kp = 0;
        double mg = INFINITY;
        double pi[3] = {x[i], y[i], z[i]};
        for (int64_t s = nb->off[i]; s < nb->off[i + 1]; ++s) {
            int64_t j = nb->idx[s];
            double pj[3] = {x[j], y[j], z[j]};
            int b[3]; double m;
            int ok = pair_features(pi, nrm + 3 * i, pj, nrm + 3 * j, b, &m);
            if (m < mg) mg = m;
            if (!ok) continue;
            ++kp;
            cnt[b[0]]++; cnt[NB + b[1]]++; cnt[2 * NB + b[2]]++;
        }
        for (int c = 0; c < FD; ++c) spfh[FD * i + c] = kp > 0 ? (double)cnt[c] / (double)kp : 0.0;
        k[i] = (int32_t)(nb->off[i + 1] - nb->off[i]);
        kprime[i] = (int32_t)kp;
        margin[i] = mg;
    }
}

void orc_spfh(const float *x, const float *y, const float *z, const double *nrm, int64_t n,
              float r_f, double *spfh, int32_t *k, int32_t *kprime, double *margin) {
    csr_t nb = csr_build(x, y, z, n, (double)r_f);
    spfh_core(x, y, z, nrm, n, &nb, spfh, k, kprime, margin);
    csr_free(&nb);
}

/* ------------------------------------------------------------------------ */
/* O4: FPFH_i = SPFH_i + (1/k_i) sum_j SPFH_j / w_ij, w_ij = |p_j - p_i|,    */
/* then each 11-bin block is scaled to unit sum.  Valid iff k_i >= 1 and     */
/* every block has positive mass.  desc_margin = min of the SPFH margins of  */
/* i and of all its neighbours (every decision the descriptor depends on).   */
/* ------------------------------------------------------------------------ */
void orc_fpfh(const float *x, const float *y, const float *z, const double *nrm, int64_t n,
              float r_f, double *F, int32_t *valid, double *spfh_margin, double *desc_margin) {
    csr_t nb = csr_build(x, y, z, n, (double)r_f);
    double *spfh = (double *)malloc(sizeof(double) * FD * (size_t)(n > 0 ? n : 1));
    int32_t *k = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *kp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    spfh_core(x, y, z, nrm, n, &nb, spfh, k, kp, spfh_margin);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double acc[FD] = {0};
        double mg = spfh_margin[i];
        int64_t ki = nb.off[i + 1] - nb.off[i];
        for (int64_t s = nb.off[i]; s < nb.off[i + 1]; ++s) {
            int64_t j = nb.idx[s];
            double w = sqrt(dist2(x[i], y[i], z[i], x[j], y[j], z[j]));
            for (int c = 0; c < FD; ++c) acc[c] += spfh[FD * j + c] / w;
            if (spfh_margin[j] < mg) mg = spfh_margin[j];
        }
        double f[FD];
        for (int c = 0; c < FD; ++c) f[c] = spfh[FD * i + c] + (ki > 0 ? acc[c] / (double)ki : 0.0);
        int ok = ki >= 1;
        for (int blk = 0; blk < 3; ++blk) {
            double sum = 0;
            for (int c = 0; c < NB; ++c) sum += f[NB * blk + c];
            if (sum > 0) for (int c = 0; c < NB; ++c) f[NB * blk + c] /= sum;
            else ok = 0;
        }
        for (int c = 0; c < FD; ++c) F[FD * i + c] = ok ? f[c] : 0.0;
        valid[i] = ok;
        desc_margin[i] = mg;
    }
    free(spfh); free(k); free(kp);
    csr_free(&nb);
}

/* ------------------------------------------------------------------------ */
/* O5: feature-space nearest neighbours in both directions (Algorithm 1,     */
/* pre-matching cache, extended to the reciprocal test).                     */
/* D(i,j) = sum_c (F_i[c] - G_j[c])^2 in the difference form; argmin over    */
/* valid candidates, ties to the lowest index; the second best is kept for   */
/* the near-tie margin.                                                      */
/* ------------------------------------------------------------------------ */
static inline double desc_d2(const double *a, const double *b) {
    double s = 0;
    for (int c = 0; c < FD; ++c) { double d = a[c] - b[c]; s += d * d; }
    return s;
}

static void nn_rows(const double *A, const int32_t *vA, int64_t nA, const double *B, const int32_t *vB,
                    int64_t nB, int32_t *nn, double *d1, int32_t *nn2, double *d2) {
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nA; ++i) {
        double b1 = INFINITY, b2 = INFINITY;
        int64_t j1 = -1, j2 = -1;
        if (vA[i]) {
            for (int64_t j = 0; j < nB; ++j) {
                if (!vB[j]) continue;
                double d = desc_d2(A + FD * i, B + FD * j);
                if (d < b1) { b2 = b1; j2 = j1; b1 = d; j1 = j; }
                else if (d < b2) { b2 = d; j2 = j; }
            }
        }
        nn[i] = (int32_t)j1; d1[i] = b1; nn2[i] = (int32_t)j2; d2[i] = b2;
    }
}

void orc_match(const double *F, const int32_t *vF, int64_t nP,
               const double *G, const int32_t *vG, int64_t nQ,
               int32_t *nnQ, double *d1Q, int32_t *nn2Q, double *d2Q,
               int32_t *nnP, double *d1P, int32_t *nn2P, double *d2P) {
    nn_rows(F, vF, nP, G, vG, nQ, nnQ, d1Q, nn2Q, d2Q);
    nn_rows(G, vG, nQ, F, vF, nP, nnP, d1P, nn2P, d2P);
}

/* Near-tie margin of one candidate: the change of D(i,j) that descriptors
 * within relative tolerance eps, plus float32 re-ranking, can cause. */
static inline double tie_err(double D, double na, double nb, double eps) {
    double s = na + nb;
    return 2.0 * eps * sqrt(D) * s + eps * eps * s * s + 8.0 * FD * ldexp(1.0, -24) * D;
}

static void tie_rows(const double *A, int64_t nA, const double *B,
                     const int32_t *nn, const double *d1, const int32_t *nn2, const double *d2,
                     double eps, uint8_t *tie) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nA; ++i) {
        tie[i] = 0;
        if (nn[i] < 0 || nn2[i] < 0) continue;
        double s = 0; for (int c = 0; c < FD; ++c) s += A[FD * i + c] * A[FD * i + c];
        double na = sqrt(s);
        double n1 = 0, n2 = 0;
        for (int c = 0; c < FD; ++c) { n1 += B[FD * nn[i] + c] * B[FD * nn[i] + c]; n2 += B[FD * nn2[i] + c] * B[FD * nn2[i] + c]; }
        double e = tie_err(d1[i], na, sqrt(n1), eps) + tie_err(d2[i], na, sqrt(n2), eps);
        tie[i] = (d2[i] - d1[i]) <= e;
    }
}

void orc_tie_flags(const double *F, int64_t nP, const double *G, int64_t nQ,
                   const int32_t *nnQ, const double *d1Q, const int32_t *nn2Q, const double *d2Q,
                   const int32_t *nnP, const double *d1P, const int32_t *nn2P, const double *d2P,
                   double eps, uint8_t *tieP, uint8_t *tieQ) {
    tie_rows(F, nP, G, nnQ, d1Q, nn2Q, d2Q, eps, tieP);
    tie_rows(G, nQ, F, nnP, d1P, nn2P, d2P, eps, tieQ);
}

/* ------------------------------------------------------------------------ */
/* O6: quadruple consistency filter (Section IV, Algorithm 1: four points    */
/* picked at random from P, their cached feature neighbours in Q, and the    */
/* similar-polygon pre-rejection with tau = 0.9), used as a filter.          */
/* Counter-based randomness: the n-th output r of SplitMix64 (Steele, Lea    */
/* and Flood, 2014) with the stated seed, n = (trial << 8) | (slot << 6) |   */
/* attempt.  A draw is the P index i = ((r >> 32) N_P) >> 32, uniform over  */
/* [0, N_P); slot s keeps the first of at most 64 attempts whose i has a     */
/* reciprocal correspondence and differs from the earlier slots, else the    */
/* trial is void.  Keying the draws by P index keeps them local: whether one */
/* point has a correspondence changes only the trials that draw that point. */
/* The closed quadrilateral of the 4 points must have every squared edge     */
/* ratio within tau^2 in both directions; a zero edge rejects.  Passing      */
/* trials flag their 4 correspondences (an order-free OR).                   */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int64_t orc_consistency(const float *px, const float *py, const float *pz, int64_t nP,
                        const float *qx, const float *qy, const float *qz,
                        const int32_t *nnQ, const uint8_t *mutual, int64_t n_trials,
                        float tau, uint64_t seed, uint8_t *flag) {
    double t2 = (double)tau * (double)tau;
    memset(flag, 0, (size_t)(nP > 0 ? nP : 0));
    int64_t passed = 0;
    if (nP <= 0) return 0;
    #pragma omp parallel for schedule(static) reduction(+ : passed)
    for (int64_t t = 0; t < n_trials; ++t) {
        int64_t id[4];
        int ok = 1;
        for (int s = 0; s < 4 && ok; ++s) {
            int found = 0;
            for (int a = 0; a < 64; ++a) {
                uint64_t r = orc_splitmix64(seed, ((uint64_t)t << 8) | ((uint64_t)s << 6) | (uint64_t)a);
                int64_t i = (int64_t)(((r >> 32) * (uint64_t)nP) >> 32);
                if (!mutual[i]) continue;
                int dup = 0;
                for (int u = 0; u < s; ++u) dup |= (id[u] == i);
                if (dup) continue;
                id[s] = i; found = 1; break;
            }
            ok = found;
        }
        if (!ok) continue;
        for (int k = 0; k < 4 && ok; ++k) {
            int64_t i0 = id[k], i1 = id[(k + 1) & 3];
            int64_t j0 = nnQ[i0], j1 = nnQ[i1];
            double a = dist2(px[i0], py[i0], pz[i0], px[i1], py[i1], pz[i1]);
            double b = dist2(qx[j0], qy[j0], qz[j0], qx[j1], qy[j1], qz[j1]);
            if (a == 0.0 || b == 0.0 || a < t2 * b || b < t2 * a) ok = 0;
        }
        if (!ok) continue;
        ++passed;
        for (int k = 0; k < 4; ++k) {
            #pragma omp atomic write
            flag[id[k]] = 1;
        }
    }
    return passed;
}

/* ------------------------------------------------------------------------ */
/* O7: robust pose by graduated non-convexity.                               */
/* Energy (eq. 2 restricted to one pair, Psi of eq. 4):                       */
/*   E_mu(T, l) = sum_c l_c |R p_c + t - q_c|^2 + mu sum_c (sqrt(l_c) - 1)^2   */
/* Minimising over l gives l_c = (mu / (mu + s_c))^2 and                     */
/* E_mu(T) = sum_c mu s_c / (mu + s_c).  Gauss-Newton on T with the          */
/* linearisation of eq. 5: G_c = [ -[p'_c]x | I ], p'_c = R p_c + t,          */
/* H = sum l G^T G, g = sum l G^T r, H xi = -g (Cholesky), T <- Exp(xi) T    */
/* with Exp(xi) = [Rod(omega) | v].  mu starts at the squared diagonal of    */
/* the correspondences' bounding box and is divided by gnc_div every         */
/* gnc_every iterations down to delta^2, then polished at delta^2 until      */
/* |xi|_inf < 1e-12.                                                         */
/* ------------------------------------------------------------------------ */
static void rodrigues(const double w[3], double R[3][3]) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2), A, B;
    if (th < 1e-4) { A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0; B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0; }
    else { double sh = sin(0.5 * th); A = sin(th) / th; B = 2.0 * sh * sh / th2; }
    double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    double K2[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
        K2[i][j] = 0; for (int k = 0; k < 3; ++k) K2[i][j] += K[i][k] * K[k][j];
    }
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j)
        R[i][j] = (i == j) + A * K[i][j] + B * K2[i][j];
}

/* one Gauss-Newton step at fixed mu; returns 0 on a non-positive pivot */
static int gn_step(const double *p, const double *q, int64_t m, double R[3][3], double t[3],
                   double mu, double xi[6]) {
    double H[6][6] = {{0}}, g[6] = {0};
    for (int64_t c = 0; c < m; ++c) {
        double pp[3];
        for (int a = 0; a < 3; ++a) pp[a] = R[a][0] * p[3 * c] + R[a][1] * p[3 * c + 1] + R[a][2] * p[3 * c + 2] + t[a];
        double r[3] = {pp[0] - q[3 * c], pp[1] - q[3 * c + 1], pp[2] - q[3 * c + 2]};
        double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double l = mu / (mu + s); l = l * l;
        /* G = [ -[p']x | I ] (3x6) */
        double G[3][6] = {{0, pp[2], -pp[1], 1, 0, 0},
                          {-pp[2], 0, pp[0], 0, 1, 0},
                          {pp[1], -pp[0], 0, 0, 0, 1}};
        for (int a = 0; a < 6; ++a) {
            for (int b = 0; b < 6; ++b) H[a][b] += l * (G[0][a] * G[0][b] + G[1][a] * G[1][b] + G[2][a] * G[2][b]);
            g[a] += l * (G[0][a] * r[0] + G[1][a] * r[1] + G[2][a] * r[2]);
        }
    }
    /* Cholesky H = L L^T */
    double L[6][6] = {{0}}, tr = 0;
    for (int a = 0; a < 6; ++a) tr += H[a][a];
    for (int j = 0; j < 6; ++j) {
        double d = H[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 1e-12 * tr)) return 0;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double s = H[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s / L[j][j];
        }
    }
    double yv[6];
    for (int i = 0; i < 6; ++i) { double s = -g[i]; for (int k = 0; k < i; ++k) s -= L[i][k] * yv[k]; yv[i] = s / L[i][i]; }
    for (int i = 5; i >= 0; --i) { double s = yv[i]; for (int k = i + 1; k < 6; ++k) s -= L[k][i] * xi[k]; xi[i] = s / L[i][i]; }
    return 1;
}

static void apply_xi(double R[3][3], double t[3], const double xi[6]) {
    double D[3][3], Rn[3][3], tn[3];
    rodrigues(xi, D);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Rn[i][j] = D[i][0] * R[0][j] + D[i][1] * R[1][j] + D[i][2] * R[2][j];
        tn[i] = D[i][0] * t[0] + D[i][1] * t[1] + D[i][2] * t[2] + xi[3 + i];
    }
    memcpy(R, Rn, sizeof Rn);
    memcpy(t, tn, sizeof tn);
}

static double energy_at(const double *p, const double *q, int64_t m, double R[3][3], const double t[3], double mu) {
    double E = 0;
    for (int64_t c = 0; c < m; ++c) {
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = R[a][0] * p[3 * c] + R[a][1] * p[3 * c + 1] + R[a][2] * p[3 * c + 2] + t[a] - q[3 * c + a];
        double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        E += mu * s / (mu + s);
    }
    return E;
}

int32_t orc_gnc(const double *p, const double *q, int64_t m, const orc_params *prm,
                double *T, double *mu_final, double *energy, int32_t *iters) {
    double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, t[3] = {0, 0, 0};
    int32_t status = ORC_ACCEPTED, it = 0;
    double delta2 = (double)prm->max_corr * (double)prm->max_corr;
    double mu = delta2;
    if (m < 3) status = ORC_DEGENERATE;
    else {
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t c = 0; c < m; ++c) for (int a = 0; a < 3; ++a) {
            double u = p[3 * c + a], v = q[3 * c + a];
            mn[a] = fmin(mn[a], fmin(u, v));
            mx[a] = fmax(mx[a], fmax(u, v));
        }
        mu = (mx[0] - mn[0]) * (mx[0] - mn[0]) + (mx[1] - mn[1]) * (mx[1] - mn[1]) + (mx[2] - mn[2]) * (mx[2] - mn[2]);
        double xi[6];
        int anneal = 0;
        while (mu > delta2 && anneal < prm->gnc_max_iter) {
            if (!gn_step(p, q, m, R, t, mu, xi)) { status = ORC_DEGENERATE; break; }
            apply_xi(R, t, xi);
            ++anneal; ++it;
            if (anneal % prm->gnc_every == 0) { mu /= prm->gnc_div; if (mu < delta2) mu = delta2; }
        }
        if (status != ORC_DEGENERATE) {
            mu = delta2;
            for (int k = 0; k < prm->polish_iter; ++k) {
                if (!gn_step(p, q, m, R, t, mu, xi)) { status = ORC_DEGENERATE; break; }
                apply_xi(R, t, xi);
                ++it;
                double mxi = 0;
                for (int a = 0; a < 6; ++a) if (fabs(xi[a]) > mxi) mxi = fabs(xi[a]);
                if (mxi < 1e-12) break;
            }
        }
    }
    for (int i = 0; i < 16; ++i) T[i] = 0;
    for (int i = 0; i < 3; ++i) { for (int j = 0; j < 3; ++j) T[4 * i + j] = R[i][j]; T[4 * i + 3] = t[i]; }
    T[15] = 1;
    *mu_final = mu;
    *energy = m > 0 ? energy_at(p, q, m, R, t, mu) : 0.0;
    *iters = it;
    return status;
}

/* one row of a rigid transform applied to (x, y, z) with offset c, in the    */
/* pinned order c + r0 x, then + r1 y, then + r2 z, each step one fma        */
static inline double xform_row(const double *r, double x, double y, double z, double c) {
    return fma(r[2], z, fma(r[1], y, fma(r[0], x, c)));
}

/* ------------------------------------------------------------------------ */
/* O8: verification (Section IV, Algorithm 1's hypothesis test: inlier     */
/* ratio and fitness; 3D grid search of eq. 1).  Inlier: the nearest q       */
/* within delta of T p (optionally with normal agreement (R n_p) . n_q >=    */
/* cos).  T p and R n_p use the pinned fma order of xform_row, so the        */
/* predicate is a function of the inputs alone.  ratio = inliers / N_P,      */
/* fitness = RMS distance of inliers to their nearest q.                     */
/* ------------------------------------------------------------------------ */
/* Squared distance from T p_i to its nearest q_j within delta (with the
 * normal check when asked), or INFINITY when there is none; g is Q's grid
 * with cell >= delta. */
static double inlier_d2(const ogrid *g, const float *px, const float *py, const float *pz, const double *nP_,
                        int64_t i, const float *qx, const float *qy, const float *qz, const double *nQ_,
                        const double *T, double d2max, int32_t normal_check, double cth,
                        int64_t **tmp, int64_t *cap) {
    double p[3] = {px[i], py[i], pz[i]}, tp[3];
    for (int a = 0; a < 3; ++a) tp[a] = xform_row(T + 4 * a, p[0], p[1], p[2], T[4 * a + 3]);
    int64_t k = grid_query(g, qx, qy, qz, tp[0], tp[1], tp[2], d2max, -1.0, *tmp, *cap);
    while (k > *cap) { *cap = 2 * k; *tmp = (int64_t *)realloc(*tmp, sizeof(int64_t) * (size_t)*cap);
                       k = grid_query(g, qx, qy, qz, tp[0], tp[1], tp[2], d2max, -1.0, *tmp, *cap); }
    double best = INFINITY;
    for (int64_t s = 0; s < k; ++s) {
        int64_t j = (*tmp)[s];
        if (normal_check) {
            const double *ni = nP_ + 3 * i, *nj = nQ_ + 3 * j;
            double rn[3];
            for (int a = 0; a < 3; ++a) rn[a] = xform_row(T + 4 * a, ni[0], ni[1], ni[2], 0.0);
            if (fma(rn[2], nj[2], fma(rn[1], nj[1], rn[0] * nj[0])) < cth) continue;
        }
        double d2 = dist2(tp[0], tp[1], tp[2], qx[j], qy[j], qz[j]);
        if (d2 < best) best = d2;
    }
    return best <= d2max ? best : INFINITY;
}

void orc_verify(const float *px, const float *py, const float *pz, const double *nP_, int64_t nP,
                const float *qx, const float *qy, const float *qz, const double *nQ_, int64_t nQ,
                const double *T, float delta, int32_t normal_check, float normal_cos,
                int64_t *n_inliers, double *ratio, double *fitness) {
    ogrid g; grid_build(&g, qx, qy, qz, nQ, (double)delta);
    double d2max = (double)delta * (double)delta, cth = (double)normal_cos;
    int64_t cnt = 0; double ss = 0;
    #pragma omp parallel reduction(+ : cnt, ss)
    {
        int64_t cap = 4096; int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * cap);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < nP; ++i) {
            double best = inlier_d2(&g, px, py, pz, nP_, i, qx, qy, qz, nQ_, T, d2max, normal_check, cth, &tmp, &cap);
            if (best <= d2max) { cnt += 1; ss += best; }
        }
        free(tmp);
    }
    grid_free(&g);
    *n_inliers = cnt;
    *ratio = nP > 0 ? (double)cnt / (double)nP : 0.0;
    *fitness = cnt > 0 ? sqrt(ss / (double)cnt) : 0.0;
}

/* Per-point inlier flags of O8 without the normal check: flag[i] = 1 when
 * some q lies within delta of T p_i (used by the loop verification's edge
 * correspondences, Sec. V). */
void orc_inliers(const float *px, const float *py, const float *pz, int64_t nP,
                 const float *qx, const float *qy, const float *qz, int64_t nQ,
                 const double *T, float delta, uint8_t *flag) {
    ogrid g; grid_build(&g, qx, qy, qz, nQ, (double)delta);
    double d2max = (double)delta * (double)delta;
    #pragma omp parallel
    {
        int64_t cap = 4096; int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * cap);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < nP; ++i)
            flag[i] = inlier_d2(&g, px, py, pz, NULL, i, qx, qy, qz, NULL, T, d2max, 0, 0.0, &tmp, &cap) <= d2max;
        free(tmp);
    }
    grid_free(&g);
}

/* ------------------------------------------------------------------------ */
/* RANSAC consensus (Section IV, Algorithm 1), the paper's own pose stage.   */
/* Hypothesis t draws four distinct points of P as the consistency filter   */
/* does (same generator and counter layout), except that a point is eligible */
/* when its descriptor has a nearest neighbour in Q (the one-directional     */
/* pre-matching cache nnQ), not only a reciprocal one.  Its correspondences  */
/* q_k = Q[nnQ(p_k)].  Pre-rejection: the similar-polygon test of O6.        */
/* Survivors get the least-squares rigid transform of their 4 pairs (Horn's  */
/* closed form with unit quaternions, 1987), then are tested on all of P:     */
/* inliers as in O8 (with the normal check, which the paper moves from       */
/* pre-rejection into this test), ratio = inliers / N_P.  The result is the  */
/* hypothesis with the most inliers; equal counts go to the smaller sum of   */
/* inlier squared distances (smaller RMS), then to the lower index.  It is   */
/* accepted when its ratio reaches min_ratio.  A fit whose largest two       */
/* quaternion eigenvalues are closer than 1e-9 of the largest magnitude      */
/* (collinear or coincident points) is rejected.                             */
/* ------------------------------------------------------------------------ */
static void jacobi4(double A[4][4], double w[4], double V[4][4]) {
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) V[i][j] = (i == j);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0, tr = 0;
        for (int p = 0; p < 4; ++p) { tr += fabs(A[p][p]); for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q]; }
        if (off == 0.0 || sqrt(off) <= 1e-18 * tr) break;
        for (int p = 0; p < 3; ++p) for (int q = p + 1; q < 4; ++q) {
            double apq = A[p][q];
            if (apq == 0.0) continue;
            double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
            double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            for (int k = 0; k < 4; ++k) {
                double akp = A[k][p], akq = A[k][q];
                A[k][p] = c * akp - s * akq;
                A[k][q] = s * akp + c * akq;
            }
            for (int k = 0; k < 4; ++k) {
                double apk = A[p][k], aqk = A[q][k];
                A[p][k] = c * apk - s * aqk;
                A[q][k] = s * apk + c * aqk;
            }
            for (int k = 0; k < 4; ++k) {
                double vkp = V[k][p], vkq = V[k][q];
                V[k][p] = c * vkp - s * vkq;
                V[k][q] = s * vkp + c * vkq;
            }
        }
    }
    for (int i = 0; i < 4; ++i) w[i] = A[i][i];
}

/* Least-squares rigid transform (R, t) with q_k ~ R p_k + t from m pairs
 * (Horn 1987).  Returns 0 when the optimal rotation is not unique. */
int32_t orc_rigid_fit(const double *p, const double *q, int64_t m, double *T) {
    double pm[3] = {0, 0, 0}, qm[3] = {0, 0, 0};
    for (int64_t k = 0; k < m; ++k) for (int a = 0; a < 3; ++a) { pm[a] += p[3 * k + a]; qm[a] += q[3 * k + a]; }
    for (int a = 0; a < 3; ++a) { pm[a] /= (double)m; qm[a] /= (double)m; }
    double S[3][3] = {{0}};
    for (int64_t k = 0; k < m; ++k)
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b)
            S[a][b] += (p[3 * k + a] - pm[a]) * (q[3 * k + b] - qm[b]);
    double N[4][4] = {
        {S[0][0] + S[1][1] + S[2][2], S[1][2] - S[2][1], S[2][0] - S[0][2], S[0][1] - S[1][0]},
        {S[1][2] - S[2][1], S[0][0] - S[1][1] - S[2][2], S[0][1] + S[1][0], S[2][0] + S[0][2]},
        {S[2][0] - S[0][2], S[0][1] + S[1][0], -S[0][0] + S[1][1] - S[2][2], S[1][2] + S[2][1]},
        {S[0][1] - S[1][0], S[2][0] + S[0][2], S[1][2] + S[2][1], -S[0][0] - S[1][1] + S[2][2]}};
    double w[4], V[4][4];
    jacobi4(N, w, V);
    int i1 = 0;
    for (int i = 1; i < 4; ++i) if (w[i] > w[i1]) i1 = i;
    double w2 = -INFINITY, wmax = 0;
    for (int i = 0; i < 4; ++i) { if (i != i1 && w[i] > w2) w2 = w[i]; if (fabs(w[i]) > wmax) wmax = fabs(w[i]); }
    for (int i = 0; i < 16; ++i) T[i] = (i % 5 == 0);
    if (!(w[i1] - w2 > 1e-9 * wmax)) return 0;
    double qw = V[0][i1], qx = V[1][i1], qy = V[2][i1], qz = V[3][i1];
    double nq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= nq; qx /= nq; qy /= nq; qz /= nq;
    double R[3][3] = {
        {qw * qw + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
        {2 * (qy * qx + qw * qz), qw * qw - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - qw * qx)},
        {2 * (qz * qx - qw * qy), 2 * (qz * qy + qw * qx), qw * qw - qx * qx - qy * qy + qz * qz}};
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) T[4 * a + b] = R[a][b];
        T[4 * a + 3] = qm[a] - (R[a][0] * pm[0] + R[a][1] * pm[1] + R[a][2] * pm[2]);
    }
    return 1;
}

/* Hypotheses and their pre-rejection: ok[t] = 1 when hypothesis t filled
 * its four slots and passed the polygon test, its P indices in mem[4 t ..]. */
void orc_ransac_hypotheses(const float *px, const float *py, const float *pz, int64_t nP,
                           const float *qx, const float *qy, const float *qz, const int32_t *nnQ,
                           int64_t n_hyp, float tau, uint64_t seed, uint8_t *ok, int64_t *mem) {
    double t2 = (double)tau * (double)tau;
    memset(ok, 0, (size_t)(n_hyp > 0 ? n_hyp : 0));
    if (nP <= 0) return;
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n_hyp; ++t) {
        int64_t id[4];
        int good = 1;
        for (int s = 0; s < 4 && good; ++s) {
            int found = 0;
            for (int a = 0; a < 64; ++a) {
                uint64_t r = orc_splitmix64(seed, ((uint64_t)t << 8) | ((uint64_t)s << 6) | (uint64_t)a);
                int64_t i = (int64_t)(((r >> 32) * (uint64_t)nP) >> 32);
                if (nnQ[i] < 0) continue;
                int dup = 0;
                for (int u = 0; u < s; ++u) dup |= (id[u] == i);
                if (dup) continue;
                id[s] = i; found = 1; break;
            }
            good = found;
        }
        for (int k = 0; k < 4 && good; ++k) {
            int64_t i0 = id[k], i1 = id[(k + 1) & 3];
            int64_t j0 = nnQ[i0], j1 = nnQ[i1];
            double a = dist2(px[i0], py[i0], pz[i0], px[i1], py[i1], pz[i1]);
            double b = dist2(qx[j0], qy[j0], qz[j0], qx[j1], qy[j1], qz[j1]);
            if (a == 0.0 || b == 0.0 || a < t2 * b || b < t2 * a) good = 0;
        }
        if (good) { ok[t] = 1; for (int k = 0; k < 4; ++k) mem[4 * t + k] = id[k]; }
    }
}

int32_t orc_ransac(const float *px, const float *py, const float *pz, const double *nP_, int64_t nP,
                   const float *qx, const float *qy, const float *qz, const double *nQ_, int64_t nQ,
                   const int32_t *nnQ, int64_t n_hyp, float tau, uint64_t seed, float delta,
                   int32_t normal_check, float normal_cos, float min_ratio,
                   double *T, orc_ransac_info *info) {
    memset(info, 0, sizeof *info);
    info->best = info->second = -1;
    for (int i = 0; i < 16; ++i) T[i] = (i % 5 == 0);
    if (nP <= 0) return ORC_DEGENERATE;
    double d2max = (double)delta * (double)delta, cth = (double)normal_cos;
    /* hypotheses and pre-rejection */
    int64_t *surv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_hyp > 0 ? n_hyp : 1));
    int64_t (*mem)[4] = malloc(sizeof(int64_t[4]) * (size_t)(n_hyp > 0 ? n_hyp : 1));
    uint8_t *ok = (uint8_t *)calloc((size_t)(n_hyp > 0 ? n_hyp : 1), 1);
    orc_ransac_hypotheses(px, py, pz, nP, qx, qy, qz, nnQ, n_hyp, tau, seed, ok, &mem[0][0]);
    int64_t ns = 0;
    for (int64_t t = 0; t < n_hyp; ++t) if (ok[t]) surv[ns++] = t;
    info->n_survivors = ns;
    /* fit and test every survivor */
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    double *ssum = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
    double *Ts = (double *)malloc(sizeof(double) * 16 * (size_t)(ns > 0 ? ns : 1));
    ogrid g; grid_build(&g, qx, qy, qz, nQ, (double)delta);
    int64_t nfit = 0;
    #pragma omp parallel reduction(+ : nfit)
    {
        int64_t cap = 4096; int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * cap);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t h = 0; h < ns; ++h) {
            const int64_t *id = mem[surv[h]];
            double pp[12], qq[12];
            for (int k = 0; k < 4; ++k) {
                int64_t i = id[k], j = nnQ[i];
                pp[3 * k] = px[i]; pp[3 * k + 1] = py[i]; pp[3 * k + 2] = pz[i];
                qq[3 * k] = qx[j]; qq[3 * k + 1] = qy[j]; qq[3 * k + 2] = qz[j];
            }
            double *Th = Ts + 16 * h;
            cnt[h] = -1; ssum[h] = 0;
            if (!orc_rigid_fit(pp, qq, 4, Th)) continue;
            ++nfit;
            int64_t c = 0; double sd = 0;
            for (int64_t i = 0; i < nP; ++i) {
                double d2 = inlier_d2(&g, px, py, pz, nP_, i, qx, qy, qz, nQ_, Th, d2max, normal_check, cth, &tmp, &cap);
                if (d2 <= d2max) { ++c; sd += d2; }
            }
            cnt[h] = c; ssum[h] = sd;
        }
        free(tmp);
    }
    grid_free(&g);
    info->n_fitted = nfit;
    /* best: most inliers, then smaller squared-distance sum, then lower index */
    int64_t b1 = -1, b2 = -1;
    for (int64_t h = 0; h < ns; ++h) {
        if (cnt[h] < 0) continue;
        int better1 = b1 < 0 || cnt[h] > cnt[b1] || (cnt[h] == cnt[b1] && ssum[h] < ssum[b1]);
        if (better1) { b2 = b1; b1 = h; continue; }
        int better2 = b2 < 0 || cnt[h] > cnt[b2] || (cnt[h] == cnt[b2] && ssum[h] < ssum[b2]);
        if (better2) b2 = h;
    }
    int32_t status = ORC_DEGENERATE;
    if (b1 >= 0) {
        memcpy(T, Ts + 16 * b1, sizeof(double) * 16);
        info->best = surv[b1];
        info->n_inliers = cnt[b1];
        info->ratio = (double)cnt[b1] / (double)nP;
        info->fitness = cnt[b1] > 0 ? sqrt(ssum[b1] / (double)cnt[b1]) : 0.0;
        info->sum_d2 = ssum[b1];
        status = info->ratio >= (double)min_ratio ? ORC_ACCEPTED : ORC_REJECTED;
        if (b2 >= 0) { info->second = surv[b2]; info->second_inliers = cnt[b2]; info->second_sum_d2 = ssum[b2]; }
    }
    free(surv); free(mem); free(ok); free(cnt); free(ssum); free(Ts);
    return status;
}

/* ------------------------------------------------------------------------ */
/* O9: E = sum_c mu s_c / (mu + s_c), s_c = |R p_c + t - q_c|^2, and its      */
/* adjoint.  dE/ds = (mu/(mu+s))^2 = l_c, so                                 */
/*   dE/dp_c = 2 l_c R^T r_c,  dE/dq_c = -2 l_c r_c,                          */
/*   dE/dxi  = sum_c 2 l_c [ p'_c x r_c ; r_c ]  (left perturbation).         */
/* ------------------------------------------------------------------------ */
double orc_align_loss(const double *p, const double *q, int64_t m, const double *T, double mu,
                      double *dp, double *dq, double *dxi) {
    double E = 0, gx[6] = {0};
    for (int64_t c = 0; c < m; ++c) {
        double pp[3], r[3];
        for (int a = 0; a < 3; ++a) {
            pp[a] = T[4 * a] * p[3 * c] + T[4 * a + 1] * p[3 * c + 1] + T[4 * a + 2] * p[3 * c + 2] + T[4 * a + 3];
            r[a] = pp[a] - q[3 * c + a];
        }
        double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double l = mu / (mu + s); l = l * l;
        E += mu * s / (mu + s);
        if (dp) for (int a = 0; a < 3; ++a) dp[3 * c + a] = 2.0 * l * (T[a] * r[0] + T[4 + a] * r[1] + T[8 + a] * r[2]);
        if (dq) for (int a = 0; a < 3; ++a) dq[3 * c + a] = -2.0 * l * r[a];
        double cr[3] = {pp[1] * r[2] - pp[2] * r[1], pp[2] * r[0] - pp[0] * r[2], pp[0] * r[1] - pp[1] * r[0]};
        for (int a = 0; a < 3; ++a) { gx[a] += 2.0 * l * cr[a]; gx[3 + a] += 2.0 * l * r[a]; }
    }
    if (dxi) for (int a = 0; a < 6; ++a) dxi[a] = gx[a];
    return E;
}

/* ------------------------------------------------------------------------ */
/* whole pipeline: normals -> FPFH -> reciprocal NN -> consistency -> GNC    */
/* -> verification -> accept / reject                                        */
/* ------------------------------------------------------------------------ */
void orc_default_params(orc_params *p) {
    p->r_normal = 0.025f; p->r_feature = 0.05f; p->max_corr = 0.015f; p->tau = 0.9f;
    p->n_trials = 0; p->gnc_div = 1.4; p->gnc_every = 4; p->gnc_max_iter = 256; p->polish_iter = 32;
    p->min_inlier_ratio = 0.25f; p->min_consistent = 10; p->normal_check = 0; p->normal_cos = 0.8660254f;
    p->seed = 0x1801015720ULL;
}

int32_t orc_register_pair(const float *const *P, int64_t nP, const float *const *Q, int64_t nQ,
                          const orc_params *prm, orc_result *out,
                          int32_t *nnQ_out, uint8_t *consistent_out) {
    memset(out, 0, sizeof *out);
    for (int i = 0; i < 4; ++i) out->T[5 * i] = 1.0;
    size_t np = (size_t)(nP > 0 ? nP : 1), nq = (size_t)(nQ > 0 ? nQ : 1);
    double *nrmP = malloc(sizeof(double) * 3 * np), *nrmQ = malloc(sizeof(double) * 3 * nq);
    double *tmp1 = malloc(sizeof(double) * (np > nq ? np : nq)), *tmp2 = malloc(sizeof(double) * (np > nq ? np : nq));
    int32_t *cnt = malloc(sizeof(int32_t) * (np > nq ? np : nq));
    double *F = malloc(sizeof(double) * FD * np), *G = malloc(sizeof(double) * FD * nq);
    int32_t *vF = malloc(sizeof(int32_t) * np), *vG = malloc(sizeof(int32_t) * nq);
    int32_t *nnQ = malloc(sizeof(int32_t) * np), *nn2Q = malloc(sizeof(int32_t) * np);
    int32_t *nnP = malloc(sizeof(int32_t) * nq), *nn2P = malloc(sizeof(int32_t) * nq);
    double *d1Q = malloc(sizeof(double) * np), *d2Q = malloc(sizeof(double) * np);
    double *d1P = malloc(sizeof(double) * nq), *d2P = malloc(sizeof(double) * nq);
    uint8_t *mutual = malloc(np), *flag = malloc(np);

    orc_normals(P[0], P[1], P[2], P[3], P[4], P[5], nP, prm->r_normal, nrmP, tmp1, tmp2, cnt);
    orc_normals(Q[0], Q[1], Q[2], Q[3], Q[4], Q[5], nQ, prm->r_normal, nrmQ, tmp1, tmp2, cnt);
    orc_fpfh(P[0], P[1], P[2], nrmP, nP, prm->r_feature, F, vF, tmp1, tmp2);
    orc_fpfh(Q[0], Q[1], Q[2], nrmQ, nQ, prm->r_feature, G, vG, tmp1, tmp2);
    for (int64_t i = 0; i < nP; ++i) out->n_valid_P += vF[i];
    for (int64_t j = 0; j < nQ; ++j) out->n_valid_Q += vG[j];
    orc_match(F, vF, nP, G, vG, nQ, nnQ, d1Q, nn2Q, d2Q, nnP, d1P, nn2P, d2P);
    for (int64_t i = 0; i < nP; ++i) {
        mutual[i] = nnQ[i] >= 0 && nnP[nnQ[i]] == i;
        out->n_recip += mutual[i];
    }
    int64_t ntr = prm->n_trials > 0 ? prm->n_trials : (100 * nP < 4000000 ? 100 * nP : 4000000);
    orc_consistency(P[0], P[1], P[2], nP, Q[0], Q[1], Q[2], nnQ, mutual, ntr, prm->tau, prm->seed, flag);
    int64_t m = 0;
    for (int64_t i = 0; i < nP; ++i) m += flag[i];
    out->n_consistent = m;
    double *pc = malloc(sizeof(double) * 3 * (size_t)(m > 0 ? m : 1)), *qc = malloc(sizeof(double) * 3 * (size_t)(m > 0 ? m : 1));
    int64_t c = 0;
    for (int64_t i = 0; i < nP; ++i) if (flag[i]) {
        int64_t j = nnQ[i];
        pc[3 * c] = P[0][i]; pc[3 * c + 1] = P[1][i]; pc[3 * c + 2] = P[2][i];
        qc[3 * c] = Q[0][j]; qc[3 * c + 1] = Q[1][j]; qc[3 * c + 2] = Q[2][j];
        ++c;
    }
    out->status = orc_gnc(pc, qc, m, prm, out->T, &out->mu_final, &out->energy, &out->iters);
    orc_verify(P[0], P[1], P[2], nrmP, nP, Q[0], Q[1], Q[2], nrmQ, nQ, out->T, prm->max_corr,
               prm->normal_check, prm->normal_cos, &out->n_inliers, &out->inlier_ratio, &out->fitness);
    if (out->status != ORC_DEGENERATE) {
        int ok = m >= prm->min_consistent && out->inlier_ratio >= (double)prm->min_inlier_ratio;
        out->status = ok ? ORC_ACCEPTED : ORC_REJECTED;
    }
    if (nnQ_out) memcpy(nnQ_out, nnQ, sizeof(int32_t) * (size_t)nP);
    if (consistent_out) memcpy(consistent_out, flag, (size_t)nP);
    free(nrmP); free(nrmQ); free(tmp1); free(tmp2); free(cnt); free(F); free(G); free(vF); free(vG);
    free(nnQ); free(nn2Q); free(nnP); free(nn2P); free(d1Q); free(d2Q); free(d1P); free(d2P);
    free(mutual); free(flag); free(pc); free(qc);
    return out->status;
}
