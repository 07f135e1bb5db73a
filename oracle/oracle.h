/*
 * CPU FP64 oracle for global registration of two surface fragments
 * (LoopSmart, Sec. IV "Fast global point cloud registration on GPU",
 * Algorithm 1, and the robust line-process energy of Sec. V, eqs. 2-5).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct definition that the GPU path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  The product path never calls it and shares no code with it.
 *
 * Conventions
 *  - Clouds are float32 structure-of-arrays (x, y, z, nx, ny, nz); every
 *    computation upcasts to double first.
 *  - Float parameters are upcast to double once: r2 = (double)r * (double)r.
 *  - Squared distances use one pinned operation order,
 *      dx = (double)xj - (double)xi, ...,
 *      d2 = fma(dz, dz, fma(dy, dy, dx * dx)),
 *    so that every radius, quadruple and inlier decision is a function of the
 *    inputs alone.  The library is built with -ffp-contract=off.
 *  - Index ties are broken towards the lowest index.
 *  - Status codes: 1 accepted, 2 rejected, 3 degenerate.
 *
 * Parity pins (see tests/test_oracle_*.py): brute force on small inputs,
 * closed forms (planes, spheres, scaled copies), rigid-motion invariance,
 * recovery of a known transform, Horn/Umeyama least squares in the l == 1
 * limit, finite differences of the alignment energy.
 */
#ifndef LSR_ORACLE_H
#define LSR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ACCEPTED = 1, ORC_REJECTED = 2, ORC_DEGENERATE = 3 };

typedef struct {
    float r_normal;          /* normal-estimation radius (m) */
    float r_feature;         /* FPFH radius (m) */
    float max_corr;          /* inlier / final-kernel distance delta (m) */
    float tau;               /* polygon similarity threshold (0.9) */
    int64_t n_trials;        /* consistency trials; <= 0 -> min(4e6, 100 N_P) */
    double gnc_div;          /* mu divisor (1.4) */
    int32_t gnc_every;       /* divide mu every this many iterations (4) */
    int32_t gnc_max_iter;    /* cap on annealing iterations (256) */
    int32_t polish_iter;     /* iterations at mu = delta^2 (32) */
    float min_inlier_ratio;  /* accept threshold on the inlier ratio */
    int64_t min_consistent;  /* accept threshold on |K| */
    int32_t normal_check;    /* 1: inliers also need normal agreement */
    float normal_cos;        /* cosine threshold of the normal check */
    uint64_t seed;           /* consistency-filter RNG seed */
} orc_params;

typedef struct {
    double T[16];            /* row-major 4x4, maps P into Q's frame */
    double energy, mu_final, inlier_ratio, fitness;
    int64_t n_valid_P, n_valid_Q, n_recip, n_consistent, n_inliers;
    int32_t status, iters;
} orc_result;

/* ---- O1: radius neighbourhoods N_r(i) = { j : 0 < d2(i,j) <= r^2 } ---- */
/* CSR lists sorted by index; offsets has n+1 entries.  Returns total size or
 * -1 if cap is too small (offsets are still filled). */
int64_t orc_neighbors_grid(const float *x, const float *y, const float *z, int64_t n,
                           float r, int64_t *offsets, int64_t *idx, int64_t cap);
int64_t orc_neighbors_brute(const float *x, const float *y, const float *z, int64_t n,
                            float r, int64_t *offsets, int64_t *idx, int64_t cap);

/* ---- O0: voxel downsample (optional step) ---- */
/* Returns the number of voxels; out arrays need n entries each. */
int64_t orc_voxel(const float *x, const float *y, const float *z,
                  const float *nx, const float *ny, const float *nz, int64_t n, float v,
                  float *ox, float *oy, float *oz, float *onx, float *ony, float *onz);

/* ---- O2: normals (3n interleaved doubles), eigen gap and orientation ---- */
void orc_normals(const float *x, const float *y, const float *z,
                 const float *nx, const float *ny, const float *nz, int64_t n, float r_n,
                 double *nrm, double *gap, double *orient, int32_t *count);

/* ---- O3/O4: SPFH and FPFH (33 doubles per point) ---- */
void orc_spfh(const float *x, const float *y, const float *z, const double *nrm, int64_t n,
              float r_f, double *spfh, int32_t *k, int32_t *kprime, double *margin);
void orc_fpfh(const float *x, const float *y, const float *z, const double *nrm, int64_t n,
              float r_f, double *F, int32_t *valid, double *spfh_margin, double *desc_margin);

/* ---- O5: reciprocal nearest neighbours in descriptor space ---- */
void orc_match(const double *F, const int32_t *vF, int64_t nP,
               const double *G, const int32_t *vG, int64_t nQ,
               int32_t *nnQ, double *d1Q, int32_t *nn2Q, double *d2Q,
               int32_t *nnP, double *d1P, int32_t *nn2P, double *d2P);
/* near-tie flags of rows (P) and columns (Q) for descriptor tolerance eps */
void orc_tie_flags(const double *F, int64_t nP, const double *G, int64_t nQ,
                   const int32_t *nnQ, const double *d1Q, const int32_t *nn2Q, const double *d2Q,
                   const int32_t *nnP, const double *d1P, const int32_t *nn2P, const double *d2P,
                   double eps, uint8_t *tieP, uint8_t *tieQ);

/* ---- O6: quadruple consistency filter ---- */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n);
int64_t orc_consistency(const float *px, const float *py, const float *pz, int64_t nP,
                        const float *qx, const float *qy, const float *qz,
                        const int32_t *nnQ, const uint8_t *mutual, int64_t n_trials,
                        float tau, uint64_t seed, uint8_t *flag);

/* ---- O7: graduated non-convexity robust pose ---- */
int32_t orc_gnc(const double *p, const double *q, int64_t m, const orc_params *prm,
                double *T, double *mu_final, double *energy, int32_t *iters);

/* ---- O8: verification ---- */
void orc_verify(const float *px, const float *py, const float *pz, const double *nP_, int64_t nP,
                const float *qx, const float *qy, const float *qz, const double *nQ_, int64_t nQ,
                const double *T, float delta, int32_t normal_check, float normal_cos,
                int64_t *n_inliers, double *ratio, double *fitness);

/* ---- RANSAC consensus (Algorithm 1's own pose stage) ---- */
typedef struct {
    int64_t n_survivors;     /* hypotheses that passed the polygon pre-rejection */
    int64_t n_fitted;        /* survivors with a unique least-squares rotation */
    int64_t best, second;    /* hypothesis indices of the best two (-1: none) */
    int64_t n_inliers, second_inliers;
    double ratio, fitness, sum_d2, second_sum_d2;
} orc_ransac_info;
/* Least-squares rigid transform of m point pairs (q ~ R p + t), row-major
 * 4x4; returns 0 when the rotation is not unique. */
int32_t orc_rigid_fit(const double *p, const double *q, int64_t m, double *T);
/* Hypothesis t: four P indices drawn as in O6 (eligible: nnQ >= 0) and the
 * polygon test; ok[t] (n_hyp bytes) = 1 when it survives, mem[4 t .. 4 t + 3]
 * its P indices (n_hyp x 4, set for survivors only). */
void orc_ransac_hypotheses(const float *px, const float *py, const float *pz, int64_t nP,
                           const float *qx, const float *qy, const float *qz, const int32_t *nnQ,
                           int64_t n_hyp, float tau, uint64_t seed, uint8_t *ok, int64_t *mem);
int32_t orc_ransac(const float *px, const float *py, const float *pz, const double *nP_, int64_t nP,
                   const float *qx, const float *qy, const float *qz, const double *nQ_, int64_t nQ,
                   const int32_t *nnQ, int64_t n_hyp, float tau, uint64_t seed, float delta,
                   int32_t normal_check, float normal_cos, float min_ratio,
                   double *T, orc_ransac_info *info);

/* ---- O9: robust alignment energy and its adjoint ---- */
double orc_align_loss(const double *p, const double *q, int64_t m, const double *T, double mu,
                      double *dp, double *dq, double *dxi);

/* ---- whole pipeline ---- */
void orc_default_params(orc_params *p);
int32_t orc_register_pair(const float *const *P, int64_t nP, const float *const *Q, int64_t nQ,
                          const orc_params *prm, orc_result *out,
                          int32_t *nnQ_out, uint8_t *consistent_out);

/* Dense surface correction (Sec. VI, eq. 7; surfel.c).  Pinhole camera
 * shared by the keyframes; poses are row-major 4x4 camera-to-world. */
typedef struct {
    double fx, fy, cx, cy;   /* intrinsics, pixels */
    int32_t width, height;   /* image size, pixels */
    double z_min, z_max;     /* depth range of an observation, m */
} orc_camera;

/* Moves each surfel by the mean pose correction of the keyframes that observe
 * it inside its time window t0 < t_kf < tu, rotates its normal likewise, and
 * removes the surfels no keyframe of their window observes.  Outputs are
 * compacted in input order (room for n); new_index[s] is the output slot of
 * surfel s or -1; k_obs[s] = |F|.  Returns the number kept. */
int64_t orc_surfel_correct(const float *x, const float *y, const float *z, const float *nx, const float *ny,
                           const float *nz, const int32_t *t0, const int32_t *tu, int64_t n,
                           const double *T_old, const double *T_new, const int32_t *t_kf, int32_t n_kf,
                           const orc_camera *cam, float *ox, float *oy, float *oz, float *onx, float *ony,
                           float *onz, int32_t *new_index, int32_t *k_obs);

/* Per-point inlier flags of the verification predicate (no normal check):
 * flag[i] = 1 when some q lies within delta of T p_i. */
void orc_inliers(const float *px, const float *py, const float *pz, int64_t nP,
                 const float *qx, const float *qy, const float *qz, int64_t nQ,
                 const double *T, float delta, uint8_t *flag);

/* Loop verification by a line-process pose graph (Sec. V, eqs. 2-5;
 * posegraph.c).  An edge: T maps fragment i's frame into fragment j's. */
typedef struct {
    int32_t i, j;
    double T[16];
} orc_edge;

typedef struct {
    double lambda;           /* odometry weight (paper: 1000) */
    double tau;              /* distance threshold, m (paper: 0.2); mu = tau^2 |K_loop| */
    double l_min;            /* reject when l < l_min (paper: 0.25) */
    double tol;              /* stop when |delta|_inf < tol */
    int32_t max_iter;
} orc_loop_params;

typedef struct {
    double l;                /* line process of the loop edge at the returned poses */
    double f_loop;           /* loop-edge energy xi^T Lambda xi there */
    double energy;           /* E(T) with l eliminated */
    double mu;
    int32_t status;          /* accepted (l >= l_min), rejected, degenerate (singular system) */
    int32_t iters;
} orc_loop_result;

/* Lambda (36 doubles, row-major) = sum of G_p^T G_p over the points p of
 * fragment i with a point of fragment j within eps of A p; count = |K|. */
void orc_edge_info(const float *ix, const float *iy, const float *iz, int64_t ni, const float *jx, const float *jy,
                   const float *jz, int64_t nj, const double *A, float eps, double *Lambda, int64_t *count);

/* One loop candidate against a chain of n fragments: odometry edges odo[s]
 * (n - 1, edge s joins s and s + 1 in either direction) with information
 * L_odo (36 each), the loop edge with L_loop and its correspondence count.
 * T_out: the n optimised poses (node 0 fixed at T_init[0]). */
int32_t orc_loop_solve(int32_t n, const double *T_init, const orc_edge *odo, const double *L_odo,
                       const orc_edge *loop, const double *L_loop, int64_t count_loop, const orc_loop_params *prm,
                       double *T_out, orc_loop_result *res);

#ifdef __cplusplus
}
#endif
#endif
