/*
 * lsr: global registration of two surface fragments on MI355X (gfx950).
 *
 * Problem (LoopSmart, Sec. IV): given two fragments P and Q, each a set of
 * points with normals, return the rigid transform T_QP that aligns P to Q
 * (q ~ R p + t) if they can be aligned, starting from T_QP = I (Algorithm 1).
 * The path: radius neighbourhoods on a 3-D grid (Sec. IV, eq. 1) ->
 * normals -> FPFH descriptors (the descriptor Algorithm 1 computes) ->
 * reciprocal nearest neighbours in descriptor space (Algorithm 1's
 * pre-matching cache, both directions) -> quadruple edge-ratio consistency
 * (Algorithm 1's pre-rejection, tau = 0.9) -> robust pose by graduated
 * non-convexity on the line-process energy of Sec. V (eqs. 2-5: 6x6 normal
 * equations with G = [-[p]x | I], solved in FP64) -> verification by inlier
 * ratio and fitness on the grid (Algorithm 1's hypothesis test) ->
 * accepted / rejected.
 *
 * Memory and streams
 *  - Every pointer argument marked "device" is GPU memory owned by the
 *    caller; "host" pointers are read before the call returns.
 *  - Clouds are float32 structure-of-arrays: six arrays x, y, z, nx, ny, nz
 *    of n entries each.  Normals are the fragment's input normals (used to
 *    orient the estimated normals).  Coordinates should be finite: a fragment
 *    with a non-finite coordinate is indexed with a single grid cell (results
 *    stay exact, neighbour searches cost O(n^2) for that fragment).
 *  - All calls enqueue work on `stream` (a hipStream_t; NULL means the
 *    default stream) and return without waiting.  Outputs are valid once the
 *    caller synchronises the stream.
 *  - The context owns all scratch memory.  Scratch grows on demand outside
 *    stream capture; while the stream is being captured it never allocates.
 *  - One context may be used from one host thread at a time.
 *
 * Errors: every int-returning call returns LSR_OK (0) or a negative code.
 * LSR_EINVAL: a null pointer, a size out of range, a non-finite parameter;
 * LSR_ENOMEM: scratch cannot be allocated (or would have to be during
 * capture); LSR_EHIP: a HIP runtime error.  lsr_last_error() describes the
 * last failure.  A pair that cannot be aligned is not an error: its result
 * has status LSR_REJECTED or LSR_DEGENERATE.
 */
#ifndef LSR_H
#define LSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSR_OK        0
#define LSR_EINVAL   (-1)
#define LSR_ENOMEM   (-2)
#define LSR_EHIP     (-3)

#define LSR_ACCEPTED   1
#define LSR_REJECTED   2
#define LSR_DEGENERATE 3

/* descriptor matching arithmetic */
#define LSR_FP32        0   /* exact float32 difference-form scan */
#define LSR_BF16_SCREEN 1   /* bf16 matrix-core screen, certified float32 re-rank */

typedef struct lsr_ctx lsr_ctx;

typedef struct {
    const float *x, *y, *z;      /* device, n entries each */
    const float *nx, *ny, *nz;   /* device, input normals */
    int64_t n;
} lsr_cloud;

typedef struct {
    float r_normal;          /* normal-estimation radius, m (Sec. IV uses 2x the leaf) */
    float r_feature;         /* FPFH radius, m (Sec. IV uses 5x the leaf) */
    float max_corr;          /* inlier distance delta and final kernel scale, m */
    float tau;               /* polygon similarity threshold (Sec. IV: 0.9) */
    int64_t n_trials;        /* consistency trials per pair; <= 0: min(4e6, 100 N_P) */
    double gnc_div;          /* mu divisor of the non-convexity schedule */
    int32_t gnc_every;       /* iterations per mu step */
    int32_t gnc_max_iter;    /* cap on annealing iterations */
    int32_t polish_iter;     /* iterations at mu = max_corr^2 */
    float min_inlier_ratio;  /* acceptance: inliers / N_P */
    int64_t min_consistent;  /* acceptance: minimum consistent correspondences */
    int32_t normal_check;    /* 1: an inlier also needs normal agreement */
    float normal_cos;        /* cosine threshold of the normal check */
    int32_t precision;       /* LSR_FP32 or LSR_BF16_SCREEN */
    uint64_t seed;           /* consistency-trial generator seed */
} lsr_params;

typedef struct {
    double T[16];            /* row-major 4x4, maps P into Q's frame */
    double energy;           /* robust energy at the returned pose, mu = mu_final */
    double mu_final;
    double inlier_ratio;     /* inliers / N_P */
    double fitness;          /* RMS distance of inliers */
    int64_t n_valid_P, n_valid_Q;   /* points with a valid descriptor */
    int64_t n_recip;         /* reciprocal correspondences */
    int64_t n_consistent;    /* correspondences kept by the consistency filter */
    int64_t n_inliers;
    int64_t n_fallback_rows; /* bf16 screen rows re-scanned exactly */
    int64_t n_screen_chunks; /* bf16 screen: (64-query group, 128-row chunk) visits a full sweep makes (0: FP32) */
    int64_t n_screen_chunks_swept; /* visits the screen made (its centroid passes included); below
                                      n_screen_chunks when it skips chunks */
    int32_t status;          /* LSR_ACCEPTED / LSR_REJECTED / LSR_DEGENERATE */
    int32_t iters;           /* pose iterations run */
} lsr_result;

/* Context for one device.  workspace_cap_bytes bounds the device scratch the
 * context holds at once (0: no bound).  Scratch is cached per call signature
 * (sizes, addresses, parameters); when a call needs a new block and the cap
 * would be exceeded, cached blocks are released, least recently used first
 * (after a device synchronisation); a call whose own scratch exceeds the cap
 * fails with LSR_ENOMEM and enqueues nothing.  Returns LSR_OK and *ctx, or an
 * error (LSR_EINVAL: no such device). */
int lsr_create(lsr_ctx **ctx, int device, size_t workspace_cap_bytes);
void lsr_destroy(lsr_ctx *ctx);
/* Text of the last error on this context (never NULL). */
const char *lsr_last_error(const lsr_ctx *ctx);
/* Defaults: r_normal 0.025, r_feature 0.05, max_corr 0.015, tau 0.9,
 * n_trials auto, gnc_div 1.4, gnc_every 4, gnc_max_iter 256, polish_iter 32,
 * min_inlier_ratio 0.25, min_consistent 10, normal check off (cos 30 deg),
 * precision LSR_FP32.  Algorithm 1 leaves the acceptance threshold open:
 * 0.25 maximises TPR - FPR over seeded held-out loop-closure pairs (a pair
 * counts as good when its pose is within 0.2 m RMS of the generating
 * transform over P's points). */
void lsr_default_params(lsr_params *p);

/*
 * Register one fragment pair (Algorithm 1 and Sec. IV's problem
 * statement).  P and Q: device clouds with n >= 1 points.  d_out: device
 * pointer to one lsr_result.  Deterministic: the same inputs give the same
 * bits.
 */
int lsr_register_pair(lsr_ctx *ctx, const lsr_cloud *P, const lsr_cloud *Q,
                      const lsr_params *prm, lsr_result *d_out, void *stream);

/*
 * Register n_pairs fragment pairs of uneven sizes in one batched launch
 * sequence (captured once into a HIP graph and replayed while the inputs'
 * addresses and sizes are unchanged).  P_all / Q_all: device clouds holding
 * every pair's fragment back to back; pair b's P is entries
 * [offP[b], offP[b+1]) of P_all, its Q is [offQ[b], offQ[b+1]) of Q_all.
 * offP, offQ: host arrays of n_pairs + 1 non-decreasing offsets.
 * d_out: device array of n_pairs results.  Result b equals what
 * lsr_register_pair returns for pair b alone.
 */
int lsr_register_batch(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all,
                       const int64_t *offP, const int64_t *offQ, int32_t n_pairs,
                       const lsr_params *prm, lsr_result *d_out, void *stream);

/*
 * Per-point intermediate results of a registration (Algorithm 1's feature
 * neighbour cache, the reciprocal test and the polygon filter), in the
 * caller's point order; device arrays, each may be NULL:
 *   nnQ[i]        (total P points, int32) descriptor nearest neighbour of
 *                 P point i in its pair's Q (index within that Q), -1 when
 *                 the descriptor is invalid
 *   nnP[j]        (total Q points, int32) likewise for Q points, in P
 *   mutual[i]     (total P points, uint8) 1 when nnP[nnQ[i]] = i
 *   consistent[i] (total P points, uint8) 1 when the correspondence of P
 *                 point i was kept by the consistency filter
 *   desc_P/desc_Q, valid_P/valid_Q: the descriptors the matcher compared
 */
typedef struct {
    int32_t *nnQ;
    int32_t *nnP;
    uint8_t *mutual;
    uint8_t *consistent;
    float *desc_P;               /* (total P points x 33 float32) FPFH descriptor of each P point, row-major,
                                    zero for an invalid descriptor */
    float *desc_Q;               /* (total Q points x 33) likewise */
    int32_t *valid_P;            /* (total P points) 1 when the descriptor is valid */
    int32_t *valid_Q;            /* (total Q points) likewise */
} lsr_trace;

/*
 * lsr_register_batch, then the per-point intermediate results of the run
 * into *tr (which may not be NULL; its arrays may).  The results in d_out
 * are those of lsr_register_batch.  For checks of a full run stage by stage.
 */
int lsr_register_batch_trace(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all,
                             const int64_t *offP, const int64_t *offQ, int32_t n_pairs,
                             const lsr_params *prm, lsr_result *d_out, const lsr_trace *tr,
                             void *stream);

/*
 * Robust alignment energy (eq. 2 with l eliminated, Psi of eq. 4):
 *   E = sum_c mu s_c / (mu + s_c),  s_c = |R p_c + t - q_c|^2,
 * for n_problems independent problems.  Problem k uses correspondences
 * [coff[k], coff[k+1]) of d_corr (device int32 pairs (i, j): P index, Q
 * index into P_xyz / Q_xyz, device float32 SoA x, y, z of nP / nQ points;
 * a pair with an index out of range contributes nothing), pose d_T[16 k ...]
 * (device, row-major 4x4 doubles) and d_mu[k] (device).  Writes d_E[k]
 * (device doubles).  coff: host array of n_problems + 1 offsets.
 */
int lsr_align_loss(lsr_ctx *ctx, const float *const P_xyz[3], int64_t nP,
                   const float *const Q_xyz[3], int64_t nQ, const int32_t *d_corr, const int64_t *coff, int32_t n_problems,
                   const double *d_T, const double *d_mu, double *d_E, void *stream);

/*
 * Adjoint of lsr_align_loss, scaled by d_dE[k] (device doubles).  The weights
 * l_c = (mu/(mu+s_c))^2 are recomputed, not stored.
 *   dP[i] += dE 2 l_c R^T r_c, dQ[j] += -dE 2 l_c r_c     (float32, device SoA, caller zeroes)
 *   d_dxi[6 k ...] = dE sum_c 2 l_c [p'_c x r_c ; r_c]     (left se(3) perturbation
 *                                                          T <- Exp(xi) T, xi = (omega, v))
 * A point shared by several correspondences receives the FP64 sum of their
 * contributions in ascending correspondence order, rounded once: results do
 * not depend on scheduling.
 */
int lsr_align_loss_backward(lsr_ctx *ctx, const float *const P_xyz[3], int64_t nP,
                            const float *const Q_xyz[3], int64_t nQ, const int32_t *d_corr, const int64_t *coff, int32_t n_problems,
                            const double *d_T, const double *d_mu, const double *d_dE,
                            float *const dP_xyz[3], float *const dQ_xyz[3], double *d_dxi,
                            void *stream);

/*
 * The pose retraction T <- [Rod(w) | v] T (xi = (w, v), Rod the rotation of
 * the rotation vector w) under which lsr_align_loss_backward's d_dxi is the
 * gradient at xi = 0, for n poses: d_T_out[16 k ..] = Exp(xi_k) d_T[16 k ..]
 * (device, row-major 4x4 doubles; d_xi device n x 6).
 */
int lsr_se3_retract(lsr_ctx *ctx, int32_t n, const double *d_xi, const double *d_T, double *d_T_out, void *stream);

/*
 * Chain rule through the retraction: given d_g_left (device n x 6), the
 * gradient of an energy with respect to a left perturbation of
 * Exp(xi) T (lsr_align_loss_backward's d_dxi at that pose), writes d_g_xi
 * (device n x 6), the gradient with respect to xi itself:
 * dE/dw = J_l(w)^T (g_w - v x g_v), dE/dv = g_v, with J_l the left Jacobian
 * of SO(3) (Rod(w + dw) = Rod(J_l(w) dw) Rod(w) to first order).
 */
int lsr_se3_retract_grad(lsr_ctx *ctx, int32_t n, const double *d_xi, const double *d_g_left, double *d_g_xi,
                         void *stream);

/*
 * Voxel downsampling of one cloud (Algorithm 1's first step, leaf size of
 * Sec. IV): one output point per occupied voxel floor(coord / voxel) - the
 * mean position and the normalised mean input normal (the first point's
 * normal when that mean vanishes) - ordered by ascending (kx, ky, kz).
 * out: six device arrays (x, y, z, nx, ny, nz) with room for c->n points;
 * *d_count (device) receives the number of voxels, or -1 when a coordinate is
 * not finite or lies 2^20 voxels or more from the origin (outputs then
 * unspecified).
 */
int lsr_voxel_downsample(lsr_ctx *ctx, const lsr_cloud *c, float voxel, float *const out[6],
                         int64_t *d_count, void *stream);

/* ---- RANSAC consensus (Algorithm 1's own pose stage) ---- */

/*
 * Section IV, Algorithm 1: hypotheses of four random P points, each paired
 * with its descriptor nearest neighbour in Q (the one-directional
 * pre-matching cache); hypothesis t fills slot s = 0..3 with the first of up
 * to 64 draws i = ((r >> 32) N_P) >> 32, r the n-th SplitMix64 output of the
 * seed for n = (t << 8) | (s << 6) | attempt, whose point has a neighbour and
 * differs from the earlier slots (a slot without one voids the hypothesis).
 * Pre-rejection: every edge k -> k+1 of the closed quadrilateral must have
 * squared lengths in P and Q within tau^2 of each other (a zero edge
 * rejects).  Survivors get the least-squares rigid fit of their four pairs
 * (Horn's quaternion form; refused when the rotation is not unique) and are
 * tested on all of P: inliers have a q within max_corr of T p on Q's 3-D
 * grid (eq. 1), with the normal check (R n_p) . n_q >= normal_cos when
 * normal_check is set (the paper moves that check into hypothesis testing).
 * The best hypothesis has the most inliers, then the smaller sum of squared
 * inlier distances, then the lower index; it is accepted when inliers / N_P
 * reaches min_inlier_ratio.
 */
typedef struct {
    double T[16];            /* best hypothesis, row-major 4x4 (identity when none) */
    double inlier_ratio;     /* its inliers / N_P */
    double fitness;          /* RMS distance of its inliers */
    double sum_d2;           /* sum of its inliers' squared distances */
    int64_t n_hypotheses;    /* hypotheses drawn */
    int64_t n_survivors;     /* hypotheses that passed the polygon pre-rejection */
    int64_t n_fitted;        /* survivors with a unique least-squares rotation */
    int64_t best;            /* index of the best hypothesis, -1 when none */
    int64_t n_inliers;       /* its inlier count */
    int64_t n_valid_P, n_valid_Q;   /* lsr_ransac_pair: points with a valid descriptor (0 in the stage call) */
    int32_t status;          /* LSR_ACCEPTED / LSR_REJECTED / LSR_DEGENERATE (no survivor with a unique fit) */
    int32_t pad;
} lsr_ransac_result;

/* Optional per-survivor record (device arrays of `capacity` entries each, any
 * may be NULL; survivors beyond capacity are not recorded), in no particular
 * order.  n_inliers: -1 when the fit is not unique, -2 when testing stopped
 * early because the hypothesis could no longer reach the largest count
 * completed (it cannot be chosen); such counts are not final. */
typedef struct {
    int64_t capacity;
    int64_t *hyp;            /* hypothesis index t */
    int32_t *members;        /* 4 P indices per survivor, slot order */
    int32_t *n_inliers;
    double *sum_d2;
    double *T;               /* 16 per survivor, row-major */
} lsr_ransac_trace;

/*
 * Algorithm 1 on one pair: 3-D grid, normals, FPFH, the descriptor nearest
 * neighbour of every P point in Q (prm->precision as in registration), then
 * the RANSAC consensus above with n_hyp hypotheses (<= 0: min(4e6, 100 N_P);
 * the paper uses 4e6).  Parameters used: r_normal, r_feature, precision,
 * tau, seed, max_corr, normal_check, normal_cos, min_inlier_ratio.
 * d_out: device pointer to one lsr_ransac_result.  Deterministic.
 */
int lsr_ransac_pair(lsr_ctx *ctx, const lsr_cloud *P, const lsr_cloud *Q, const lsr_params *prm, int64_t n_hyp,
                    lsr_ransac_result *d_out, void *stream);

/*
 * The RANSAC consensus alone on injected inputs: d_nnQ (device, P->n int32)
 * the descriptor neighbour of each P point in Q (-1: none); normals (device
 * n x 3 doubles) only when prm->normal_check (else may be NULL).  Q's grid
 * uses cells of at least max_corr.  tr (may be NULL) receives the survivors.
 */
int lsr_stage_ransac(lsr_ctx *ctx, const lsr_cloud *P, const double *d_nrmP, const lsr_cloud *Q,
                     const double *d_nrmQ, const int32_t *d_nnQ, int64_t n_hyp, const lsr_params *prm,
                     lsr_ransac_result *d_out, const lsr_ransac_trace *tr, void *stream);

/* ---- dense surface correction after a loop closure (Sec. VI) ---- */

/* Pinhole camera shared by the keyframes. */
typedef struct {
    double fx, fy, cx, cy;   /* intrinsics, pixels */
    int32_t width, height;   /* image size, pixels */
    double z_min, z_max;     /* depth range of an observation, m */
} lsr_camera;

/*
 * Sec. VI, eq. 7: every surfel moves by the mean of the pose corrections
 * T_new(f) T_old(f)^-1 of the keyframes f that observe it inside its fusion
 * window t0 < t_kf(f) < tu; its normal becomes the normalised sum of
 * R_new(f) R_old(f)^-1 n (unchanged if that sum vanishes).  Surfels that no
 * keyframe of their window observes are removed; the rest keep their order.
 * A keyframe observes a surfel when its position in the keyframe's old camera
 * frame, c = R_old^T (p - t_old), has z_min <= c_z <= z_max and projects
 * into the image (0 <= fx c_x + cx c_z < width c_z, likewise y with height):
 * FP64 in a fixed operation order, so the decision depends on the inputs
 * only.  No occlusion test.
 *
 * surfels: six device float arrays (x, y, z, nx, ny, nz) of n entries;
 * d_t0, d_tu: device int32 windows (first and last update, frames).
 * Keyframes (host, read before the call returns): h_T_old, h_T_new n_kf
 * row-major 4x4 camera-to-world poses (doubles, 16 each), h_t_kf n_kf time
 * stamps in non-decreasing order (LSR_EINVAL otherwise).  out: six device
 * float arrays with room for n surfels, filled with the kept surfels in
 * input order; d_new_index (device n int32, may be NULL): each surfel's
 * output slot or -1; d_k_obs (device n int32, may be NULL): |F| per surfel;
 * *d_n_kept (device int64): surfels kept.  0 <= n < 2^31, 0 <= n_kf <= 2^20.
 * Not for stream capture (copies the keyframes from host memory).
 */
int lsr_surfel_correct(lsr_ctx *ctx, const float *const surfels[6], const int32_t *d_t0, const int32_t *d_tu,
                       int64_t n, const double *h_T_old, const double *h_T_new, const int32_t *h_t_kf,
                       int32_t n_kf, const lsr_camera *cam, float *const out[6], int32_t *d_new_index,
                       int32_t *d_k_obs, int64_t *d_n_kept, void *stream);

/* ---- loop verification by a line-process pose graph (Sec. V) ---- */

/* An edge of a fragment chain: T (row-major 4x4) maps fragment i's frame
 * into fragment j's (an odometry measurement, or a loop candidate's
 * registration: lsr_register_pair(P = fragment i, Q = fragment j)). */
typedef struct {
    int32_t i, j;
    double T[16];
} lsr_edge;

typedef struct {
    double lambda;           /* odometry weight (Sec. V: 1000) */
    double tau;              /* distance threshold, m (Sec. V: 0.2); mu = tau^2 |K_loop| */
    double l_min;            /* a loop with l < l_min is rejected (Sec. V: 0.25) */
    double tol;              /* Gauss-Newton stops when |step|_inf < tol */
    float eps;               /* correspondence distance of an edge, m (Sec. V: 0.05) */
    int32_t max_iter;        /* Gauss-Newton iterations at most */
} lsr_loop_params;

typedef struct {
    double l;                /* line process of the loop edge at the returned poses */
    double f_loop;           /* the loop edge's energy xi^T Lambda xi there */
    double energy;           /* lambda sum f_odometry + mu f_loop / (mu + f_loop) */
    double mu;               /* tau^2 |K_loop| */
    int64_t n_corr;          /* |K_loop| */
    int32_t status;          /* LSR_ACCEPTED (l >= l_min), LSR_REJECTED (also: no correspondences),
                                LSR_DEGENERATE (singular normal equations) */
    int32_t iters;
} lsr_loop_result;

/* Defaults: lambda 1000, tau 0.2, l_min 0.25, tol 1e-12, eps 0.05, max_iter 100. */
void lsr_default_loop_params(lsr_loop_params *p);

/*
 * Edge information (Sec. V, eq. 5) of n_edges edges between the fragments
 * frags[0 .. n_frags) (host array of device clouds; normals unused, may be
 * NULL): K = the points p of fragment i with a point of fragment j within
 * eps of T p (FP64, fixed operation order, on j's 3-D grid), Lambda =
 * sum_{p in K} G_p^T G_p with G_p = [-[p]x | I] (p in fragment i's frame).
 * h_edges: host, read before the call returns.  d_info: device n_edges x 36
 * doubles (row-major 6x6 each); d_count: device n_edges int64 (|K|).
 */
int lsr_edge_info(lsr_ctx *ctx, const lsr_cloud *frags, int32_t n_frags, const lsr_edge *h_edges,
                  int32_t n_edges, float eps, double *d_info, int64_t *d_count, void *stream);

/*
 * Sec. V, eqs. 2-5, for each of n_loops loop candidates independently: the
 * chain's poses T (n_nodes, fragment -> world, initial values h_T_init,
 * host) are moved to minimise lambda sum_s f_s + l f_loop + mu (sqrt(l) - 1)^2,
 * f = xi^T Lambda xi with xi the rotation vector and translation of the
 * edge's residual transform T_edge^-1 T_j^-1 T_i, mu = tau^2 |K_loop|, node 0
 * fixed; l = (mu / (mu + f_loop))^2 at the optimum.  Odometry edge s (host,
 * h_odo[s], n_nodes - 1 of them) must join nodes s and s + 1 (either
 * direction); d_info_odo: device (n_nodes - 1) x 36 (lsr_edge_info).  Loop
 * candidate c: h_loops[c] (host), d_info_loop + 36 c and d_count_loop[c]
 * (device).  Gauss-Newton with l re-evaluated at every iterate.  d_res:
 * device n_loops results; d_T_out: device n_loops x n_nodes x 16 optimised
 * poses, or NULL.  2 <= n_nodes <= 4096, n_loops >= 0.
 */
int lsr_loop_solve(lsr_ctx *ctx, int32_t n_nodes, const double *h_T_init, const lsr_edge *h_odo,
                   const double *d_info_odo, const lsr_edge *h_loops, int32_t n_loops, const double *d_info_loop,
                   const int64_t *d_count_loop, const lsr_loop_params *prm, double *d_T_out,
                   lsr_loop_result *d_res, void *stream);

/*
 * Both steps: the information of every odometry edge and loop candidate of
 * a chain of n_frags fragments (frags[s] is node s), then lsr_loop_solve.
 */
int lsr_loop_verify(lsr_ctx *ctx, const lsr_cloud *frags, int32_t n_frags, const double *h_T_init,
                    const lsr_edge *h_odo, const lsr_edge *h_loops, int32_t n_loops, const lsr_loop_params *prm,
                    double *d_T_out, lsr_loop_result *d_res, void *stream);

/* ---- autotuning of the batch driver's launch shapes ---- */

#define LSR_MAX_VARIANTS 8

/* Launch-shape choice of a context (not a parameter of the method: every
 * variant computes the same bits).  screen_shape picks the bf16 screen's
 * waves per block, query blocks per wave and rows per LDS chunk, and whether
 * it skips the partner's 128-row chunks whose centroid bound shows they
 * cannot matter (variant 5; the result's n_screen_chunks* fields count its
 * work); consistency_shape picks the trial kernel's block width.  screen_ms and
 * consistency_ms: mean time of each variant in the last lsr_autotune call
 * (the whole bf16 matching stage, and the consistency stage), in ms. */
typedef struct {
    int32_t screen_shape, consistency_shape;
    int32_t n_screen_shapes, n_consistency_shapes;
    float screen_ms[LSR_MAX_VARIANTS];
    float consistency_ms[LSR_MAX_VARIANTS];
    int32_t from_cache;      /* lsr_autotune: 1 when the choice came from the tune cache (timings zero) */
    int32_t pad;
} lsr_tune;

/*
 * Times every variant of the tuned kernels on the given batch (arguments as
 * lsr_register_batch, without the output; the screen is tuned with
 * precision LSR_BF16_SCREEN whatever prm asks) over `reps` runs each and
 * keeps the fastest in the context.  Cached plans are dropped when the
 * choice changes, so later calls capture graphs with the chosen kernels.
 * Allocates scratch and synchronises the stream; not for capture.  *out
 * (may be NULL) receives the choice and the timings.
 */
int lsr_autotune(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all, const int64_t *offP,
                 const int64_t *offQ, int32_t n_pairs, const lsr_params *prm, int32_t reps,
                 lsr_tune *out, void *stream);
/* Tune cache: a JSON file of choices keyed by the device architecture and a
 * size bucket of the batch (pairs, mean and largest fragment, each rounded
 * up to a power of two).  With a cache set, lsr_autotune first looks the
 * batch's key up and, when it is there, takes that choice without timing;
 * otherwise it times the variants and records the choice in the file
 * (rewritten whole, through a temporary file and a rename).  path NULL or
 * empty: no cache (the default).  The path is copied. */
int lsr_set_tune_cache(lsr_ctx *ctx, const char *path);

/* Current choice (timings zero); set a saved choice (LSR_EINVAL if a
 * variant index is out of range; drops cached plans when it changes). */
int lsr_get_tune(lsr_ctx *ctx, lsr_tune *out);
int lsr_set_tune(lsr_ctx *ctx, const lsr_tune *t);

/* ---- stage entry points: one stage on injected inputs (parity checks) ---- */

/* Normals (n x 3 doubles, row-major, device) of one cloud; PCA over the
 * radius-r_normal neighbourhood plus the point, oriented by the input normal. */
int lsr_stage_normals(lsr_ctx *ctx, const lsr_cloud *c, float r_normal, double *d_nrm, void *stream);

/* FPFH (n x 33 floats, device) and validity (n int32) of one cloud given its
 * normals (n x 3 doubles, device). */
int lsr_stage_fpfh(lsr_ctx *ctx, const lsr_cloud *c, const double *d_nrm, float r_feature,
                   float *d_F, int32_t *d_valid, void *stream);

/* SPFH (n x 33 floats, device, original order) and neighbour counts k_i
 * within r_feature (n int32) of one cloud given its normals. */
int lsr_stage_spfh(lsr_ctx *ctx, const lsr_cloud *c, const double *d_nrm, float r_feature,
                   float *d_spfh, int32_t *d_k, void *stream);

/* Nearest neighbours in descriptor space, both directions: d_nnQ[i] (nP int32)
 * is the index of the closest valid G row to F row i (-1 if F_i is invalid),
 * d_dQ[i] its float32 squared distance; d_nnP / d_dP likewise for G rows.
 * F: nP x 33, G: nQ x 33 floats; vF / vG: validity.  Ties go to the lowest
 * index.  d_fallback (device int64, may be NULL) receives the number of rows
 * the bf16 screen re-scanned exactly. */
int lsr_stage_match(lsr_ctx *ctx, const float *d_F, const int32_t *d_vF, int64_t nP,
                    const float *d_G, const int32_t *d_vG, int64_t nQ, int32_t precision,
                    int32_t *d_nnQ, float *d_dQ, int32_t *d_nnP, float *d_dP,
                    int64_t *d_fallback, void *stream);

/* Consistency filter on given correspondences: d_nnQ (nP int32), d_mutual
 * (nP uint8); writes d_flag (nP uint8) and d_passed (one int64: passing
 * trials).  n_trials <= 0 means min(4e6, 100 nP). */
int lsr_stage_consistency(lsr_ctx *ctx, const lsr_cloud *P, const lsr_cloud *Q,
                          const int32_t *d_nnQ, const uint8_t *d_mutual, int64_t n_trials,
                          float tau, uint64_t seed, uint8_t *d_flag, int64_t *d_passed, void *stream);

/* Robust pose from m correspondences (device m x 3 doubles p and q).
 * Writes d_T (16 doubles) and d_info = {status, iters, mu_final, energy} as
 * doubles. */
int lsr_stage_gnc(lsr_ctx *ctx, const double *d_p, const double *d_q, int64_t m,
                  const lsr_params *prm, double *d_T, double *d_info, void *stream);

/* lsr_stage_gnc for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same results, and no allocation of any kind.  The
 * solver's state (one 1 KiB block per GPU, a static device array held until
 * the process ends) is shared by every call on that GPU; calls that overlap
 * on one GPU (different streams, or different host threads) race and must be
 * serialised by the caller.  The state is written in full by each solve,
 * so no call depends on an earlier one; its size does not depend on m (the
 * correspondences are read from the caller's arrays), so no input size is
 * refused for lack of scratch.  LSR_EHIP if the array's device address
 * could not be obtained when the context was created. */
int lsr_stage_gnc_noalloc(lsr_ctx *ctx, const double *d_p, const double *d_q, int64_t m,
                          const lsr_params *prm, double *d_T, double *d_info, void *stream);

/* Verification of pose d_T (device 16 doubles): d_info = {n_inliers, ratio,
 * fitness} as doubles.  Normals (device n x 3 doubles) may be NULL when the
 * normal check is off. */
int lsr_stage_verify(lsr_ctx *ctx, const lsr_cloud *P, const double *d_nrmP,
                     const lsr_cloud *Q, const double *d_nrmQ, const double *d_T,
                     float delta, int32_t normal_check, float normal_cos,
                     double *d_info, void *stream);

/* ---- diagnostics ---- */

/* enable != 0: every following register call runs eagerly (no graph) and
 * records a HIP event on its stream after each step.  Resets the record. */
int lsr_set_timing(lsr_ctx *ctx, int enable);
/* Waits for the device, then returns the steps recorded since the last
 * call: names (host, max_steps x 32 chars, may be NULL) and durations ms
 * (host, may be NULL) of step k = time from step k-1's event to its own. */
int lsr_get_timing(lsr_ctx *ctx, int max_steps, char *names, double *ms, int *n_steps);

#ifdef __cplusplus
}
#endif
#endif
