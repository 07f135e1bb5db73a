/*
 * CPU FP64 oracle: dense surface correction after a loop closure
 * (LoopSmart, Sec. VI, eq. 7).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * A surfel observed by the keyframes F (those whose camera sees it and whose
 * time stamp lies strictly between the surfel's first and last update) moves
 * by the average of their pose corrections:
 *     p' = (1/k) sum_{f in F} T_new(f) T_old(f)^-1 p,
 *     n' = normalise( sum_{f in F} R_new(f) R_old(f)^-1 n ),   k = |F|.
 * A surfel that no keyframe of its window observes is removed; the others
 * keep their order.
 *
 * Observation (the paper says only "the surfels it can observe"): the surfel
 * position in camera f's frame under the old pose, c = R_old^T (p - t_old),
 * has depth z_min <= c_z <= z_max and projects into the image,
 * 0 <= fx c_x + cx c_z < W c_z and 0 <= fy c_y + cy c_z < H c_z (the pinhole
 * projection u = fx c_x / c_z + cx in [0, W), multiplied through by c_z > 0).
 * No occlusion test (no depth maps are part of the input).
 *
 * Operation order is pinned (the GPU path uses the same one), so every
 * observation decision is a function of the inputs alone:
 *     d = p - t_old                      (float p upcast to double)
 *     c_r = fma(R_2r, d_2, fma(R_1r, d_1, R_0r * d_0))     r = x, y, z
 *     u = fma(fx, c_x, cx * c_z),  v = fma(fy, c_y, cy * c_z)
 *     test u >= 0, u < W * c_z, v >= 0, v < H * c_z.
 * Sums run over keyframes in ascending index.
 */
#include "oracle.h"

#include <math.h>

/* camera-frame coordinates under a 4x4 row-major camera-to-world pose */
static void to_camera(const double *T, double px, double py, double pz, double c[3]) {
    double d0 = px - T[3], d1 = py - T[7], d2 = pz - T[11];
    for (int r = 0; r < 3; ++r)
        c[r] = fma(T[8 + r], d2, fma(T[4 + r], d1, T[r] * d0));
}

/* R_old^T v (same order as to_camera) */
static void rotate_back(const double *T, double v0, double v1, double v2, double c[3]) {
    for (int r = 0; r < 3; ++r)
        c[r] = fma(T[8 + r], v2, fma(T[4 + r], v1, T[r] * v0));
}

static int observes(const orc_camera *cam, const double c[3]) {
    if (!(c[2] >= cam->z_min && c[2] <= cam->z_max)) return 0;
    double u = fma(cam->fx, c[0], cam->cx * c[2]);
    double v = fma(cam->fy, c[1], cam->cy * c[2]);
    return u >= 0.0 && u < (double)cam->width * c[2] && v >= 0.0 && v < (double)cam->height * c[2];
}

int64_t orc_surfel_correct(const float *x, const float *y, const float *z, const float *nx, const float *ny,
                           const float *nz, const int32_t *t0, const int32_t *tu, int64_t n,
                           const double *T_old, const double *T_new, const int32_t *t_kf, int32_t n_kf,
                           const orc_camera *cam, float *ox, float *oy, float *oz, float *onx, float *ony,
                           float *onz, int32_t *new_index, int32_t *k_obs) {
    /* first pass: the update of every surfel, at its own index */
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double sp[3] = {0, 0, 0}, sn[3] = {0, 0, 0};
        int32_t k = 0;
        for (int32_t f = 0; f < n_kf; ++f) {
            if (!(t0[s] < t_kf[f] && t_kf[f] < tu[s])) continue;
            const double *A = T_old + 16 * f, *B = T_new + 16 * f;
            double c[3];
            to_camera(A, x[s], y[s], z[s], c);
            if (!observes(cam, c)) continue;
            /* T_new T_old^-1 p = R_new c + t_new ; R_new R_old^T n */
            double m[3];
            rotate_back(A, nx[s], ny[s], nz[s], m);
            for (int r = 0; r < 3; ++r) {
                sp[r] += B[4 * r] * c[0] + B[4 * r + 1] * c[1] + B[4 * r + 2] * c[2] + B[4 * r + 3];
                sn[r] += B[4 * r] * m[0] + B[4 * r + 1] * m[1] + B[4 * r + 2] * m[2];
            }
            ++k;
        }
        k_obs[s] = k;
        new_index[s] = k > 0;
        if (k > 0) {
            double len = sqrt(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
            ox[s] = (float)(sp[0] / k); oy[s] = (float)(sp[1] / k); oz[s] = (float)(sp[2] / k);
            if (len > 0) { onx[s] = (float)(sn[0] / len); ony[s] = (float)(sn[1] / len); onz[s] = (float)(sn[2] / len); }
            else { onx[s] = nx[s]; ony[s] = ny[s]; onz[s] = nz[s]; }
        }
    }
    /* second pass: keep the observed surfels in order */
    int64_t m = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (!new_index[s]) { new_index[s] = -1; continue; }
        ox[m] = ox[s]; oy[m] = oy[s]; oz[m] = oz[s];
        onx[m] = onx[s]; ony[m] = ony[s]; onz[m] = onz[s];
        new_index[s] = (int32_t)m++;
    }
    return m;
}
