// Dense surface correction after a loop closure (Sec. VI, eq. 7).
//
// Every surfel moves by the mean pose correction T_new T_old^-1 of the
// keyframes F that observe it inside its fusion window t0 < t_kf < tu, its
// normal by the normalised sum of the corresponding rotations; a surfel with
// no such keyframe is removed and the others keep their order.  A keyframe
// observes a surfel when the surfel's position in the old camera frame,
// c = R_old^T (p - t_old), has depth in [z_min, z_max] and projects into the
// image: 0 <= fx c_x + cx c_z < W c_z, 0 <= fy c_y + cy c_z < H c_z.  The
// decision is FP64 in one pinned operation order (explicit fma), so it is a
// function of the inputs alone; sums run over keyframes in ascending index.
//
// Layout: surfels as float SoA (x y z nx ny nz) with int32 window bounds;
// the keyframe table in device memory, per keyframe the two row-major 4x4
// poses (FP64) and the time stamp, time stamps non-decreasing.  A wavefront
// takes 64 consecutive surfels, finds each one's keyframe range by binary
// search over the time stamps (staged in LDS; the window is a contiguous
// index range when time stamps are sorted) and walks the union of its lanes'
// ranges with a wave-uniform keyframe index, so every pose is one scalar
// load shared by the wavefront, the next keyframe's fetched while the
// current one is tested.  Maps store surfels in order of first update, so
// neighbouring surfels have overlapping windows and the union stays close to
// one surfel's window.
// Pass 1 writes each surfel's update at its own index and a keep flag; an
// exclusive scan of the flags gives the output slots; pass 2 gathers the
// kept surfels in order.
#include "lsr_internal.h"

namespace lsr {

struct SurfelKf {              // device keyframe table (struct of arrays)
    const double *T_old;       // n_kf x 16
    const double *T_new;       // n_kf x 16
    const int32_t *t;          // n_kf, non-decreasing
    int32_t n;
};

__device__ __forceinline__ int first_above(const int32_t *t, int n, int32_t v) {   // first f: t[f] > v
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t[mid] > v) hi = mid; else lo = mid + 1;
    }
    return lo;
}
__device__ __forceinline__ int first_at_least(const int32_t *t, int n, int32_t v) {   // first f: t[f] >= v
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t[mid] >= v) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int KF_LDS = 4096;    // keyframe time stamps a block stages in LDS for its searches

__global__ void __launch_bounds__(256) k_surfel_update(const float *__restrict__ x, const float *__restrict__ y,
                                                       const float *__restrict__ z, const float *__restrict__ nx,
                                                       const float *__restrict__ ny, const float *__restrict__ nz,
                                                       const int32_t *__restrict__ t0, const int32_t *__restrict__ tu,
                                                       int64_t n, SurfelKf kf, lsr_camera cam,
                                                       float *__restrict__ tmp, int32_t *__restrict__ keep,
                                                       int32_t *__restrict__ k_obs) {
    __shared__ int32_t st[KF_LDS];
    const bool lds_t = kf.n <= KF_LDS;
    if (lds_t) {
        for (int k = threadIdx.x; k < kf.n; k += 256) st[k] = kf.t[k];
        __syncthreads();
    }
    const int32_t *tt = lds_t ? st : kf.t;
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = s < n;
    double p0 = 0, p1 = 0, p2 = 0, m0 = 0, m1 = 0, m2 = 0;
    int lo = kf.n, hi = 0;
    if (act) {
        p0 = x[s]; p1 = y[s]; p2 = z[s];
        m0 = nx[s]; m1 = ny[s]; m2 = nz[s];
        lo = first_above(tt, kf.n, t0[s]);
        hi = first_at_least(tt, kf.n, tu[s]);
    }
    const int wlo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    const int whi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    double sp0 = 0, sp1 = 0, sp2 = 0, sn0 = 0, sn1 = 0, sn2 = 0;
    int k = 0;
    const double W = (double)cam.width, H = (double)cam.height;
    // the old pose of the next keyframe is loaded while the current one is tested
    double A[12];
    if (wlo < whi)
        for (int q = 0; q < 12; ++q) A[q] = kf.T_old[16 * wlo + q];
    for (int f = wlo; f < whi; ++f) {
        double An[12];
        const int fn = f + 1 < whi ? f + 1 : f;
        for (int q = 0; q < 12; ++q) An[q] = kf.T_old[16 * fn + q];
        // c = R_old^T (p - t_old)
        const double d0 = p0 - A[3], d1 = p1 - A[7], d2 = p2 - A[11];
        const double c0 = __fma_rn(A[8], d2, __fma_rn(A[4], d1, A[0] * d0));
        const double c1 = __fma_rn(A[9], d2, __fma_rn(A[5], d1, A[1] * d0));
        const double c2 = __fma_rn(A[10], d2, __fma_rn(A[6], d1, A[2] * d0));
        const double u = __fma_rn(cam.fx, c0, cam.cx * c2);
        const double v = __fma_rn(cam.fy, c1, cam.cy * c2);
        const bool obs = f >= lo && f < hi && c2 >= cam.z_min && c2 <= cam.z_max && u >= 0.0 && u < W * c2 &&
                         v >= 0.0 && v < H * c2;
        if (obs) {
            const double *B = kf.T_new + 16 * f;
            // R_old^T n, then the new pose: R_new c + t_new and R_new (R_old^T n)
            const double e0 = __fma_rn(A[8], m2, __fma_rn(A[4], m1, A[0] * m0));
            const double e1 = __fma_rn(A[9], m2, __fma_rn(A[5], m1, A[1] * m0));
            const double e2 = __fma_rn(A[10], m2, __fma_rn(A[6], m1, A[2] * m0));
            sp0 += B[0] * c0 + B[1] * c1 + B[2] * c2 + B[3];
            sp1 += B[4] * c0 + B[5] * c1 + B[6] * c2 + B[7];
            sp2 += B[8] * c0 + B[9] * c1 + B[10] * c2 + B[11];
            sn0 += B[0] * e0 + B[1] * e1 + B[2] * e2;
            sn1 += B[4] * e0 + B[5] * e1 + B[6] * e2;
            sn2 += B[8] * e0 + B[9] * e1 + B[10] * e2;
            ++k;
        }
        for (int q = 0; q < 12; ++q) A[q] = An[q];
    }
    if (!act) return;
    if (k_obs) k_obs[s] = k;
    keep[s] = k > 0;
    if (k > 0) {
        const double len = sqrt(sn0 * sn0 + sn1 * sn1 + sn2 * sn2);
        tmp[s] = (float)(sp0 / k);
        tmp[n + s] = (float)(sp1 / k);
        tmp[2 * n + s] = (float)(sp2 / k);
        if (len > 0) {
            tmp[3 * n + s] = (float)(sn0 / len);
            tmp[4 * n + s] = (float)(sn1 / len);
            tmp[5 * n + s] = (float)(sn2 / len);
        } else {
            tmp[3 * n + s] = nx[s];
            tmp[4 * n + s] = ny[s];
            tmp[5 * n + s] = nz[s];
        }
    }
}

__global__ void __launch_bounds__(256) k_surfel_compact(const float *__restrict__ tmp, const int32_t *__restrict__ keep,
                                                        const int32_t *__restrict__ pos, int64_t n,
                                                        float *const *__restrict__ out, int32_t *__restrict__ new_index,
                                                        int64_t *__restrict__ n_kept) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int32_t kp = keep[s], q = pos[s];
    if (new_index) new_index[s] = kp ? q : -1;
    if (kp)
        for (int a = 0; a < 6; ++a) out[a][q] = tmp[a * n + s];
    if (s == n - 1) *n_kept = (int64_t)q + kp;
}

size_t surfel_ws_bytes(int64_t n, int32_t n_kf) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al(sizeof(float) * 6 * (size_t)n) + 2 * al(sizeof(int32_t) * (size_t)n) +
           al(sizeof(int32_t) * scan_tmp_elems(n)) + 2 * al(sizeof(double) * 16 * (size_t)n_kf) +
           al(sizeof(int32_t) * (size_t)n_kf) + 256;
}

// ws: surfel_ws_bytes(n, n_kf) bytes; the keyframe table at its end is filled by the caller (kf_*).
SurfelWs surfel_carve(char *ws, int64_t n, int32_t n_kf) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    SurfelWs w;
    size_t o = 0;
    w.tmp = (float *)(ws + o); o += al(sizeof(float) * 6 * (size_t)n);
    w.keep = (int32_t *)(ws + o); o += al(sizeof(int32_t) * (size_t)n);
    w.pos = (int32_t *)(ws + o); o += al(sizeof(int32_t) * (size_t)n);
    w.scan_tmp = (int32_t *)(ws + o); o += al(sizeof(int32_t) * scan_tmp_elems(n));
    w.T_old = (double *)(ws + o); o += al(sizeof(double) * 16 * (size_t)n_kf);
    w.T_new = (double *)(ws + o); o += al(sizeof(double) * 16 * (size_t)n_kf);
    w.t_kf = (int32_t *)(ws + o); o += al(sizeof(int32_t) * (size_t)n_kf);
    w.out_ptrs = (float **)(ws + o);
    return w;
}

hipError_t launch_surfel_correct(const float *const src[6], const int32_t *t0, const int32_t *tu, int64_t n,
                                 const SurfelWs &w, int32_t n_kf, const lsr_camera &cam, float *const *out_dev,
                                 int32_t *new_index, int32_t *k_obs, int64_t *n_kept, hipStream_t s) {
    if (n == 0) return fill<int64_t>(n_kept, 0, 1, s);
    const unsigned nb = (unsigned)((n + 255) / 256);
    SurfelKf kf{w.T_old, w.T_new, w.t_kf, n_kf};
    tmark("surfel_start", s);
    hipLaunchKernelGGL(k_surfel_update, dim3(nb), dim3(256), 0, s, src[0], src[1], src[2], src[3], src[4], src[5],
                       t0, tu, n, kf, cam, w.tmp, w.keep, k_obs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    tmark("surfel_update", s);
    if ((e = exclusive_scan_i32(w.keep, w.pos, n, w.scan_tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_surfel_compact, dim3(nb), dim3(256), 0, s, (const float *)w.tmp, (const int32_t *)w.keep,
                       (const int32_t *)w.pos, n, out_dev, new_index, n_kept);
    e = hipGetLastError();
    tmark("surfel_compact", s);
    return e;
}

}  // namespace lsr
