// Voxel downsampling (Algorithm 1's first step; leaf size of Sec. IV).
//
// key = (floor(x / v), floor(y / v), floor(z / v)) in double precision; one
// output point per occupied voxel: the mean position (double sums in
// ascending input index, rounded to float) and the normalised mean input
// normal (the first point's normal when the mean vanishes); output ordered
// by ascending (kx, ky, kz).  The three voxel indices are packed into one
// 63-bit key (21 bits each, offset 2^20) and sorted with a stable device
// radix sort, so points of a voxel stay in ascending input index.
#include <rocprim/device/device_radix_sort.hpp>

#include "lsr_internal.h"

namespace lsr {

constexpr int64_t VOX_OFF = 1 << 20;   // voxel indices must lie in [-2^20, 2^20)

__global__ void k_voxel_keys(const float *x, const float *y, const float *z, int64_t n, double v, uint64_t *keys,
                             uint32_t *idx, int32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double k[3] = {floor((double)x[i] / v), floor((double)y[i] / v), floor((double)z[i] / v)};
    uint64_t key = 0;
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        ok = ok && k[a] >= -(double)VOX_OFF && k[a] < (double)VOX_OFF;     // also false for NaN
        uint64_t u = ok ? (uint64_t)((int64_t)k[a] + VOX_OFF) : 0;
        key = (key << 21) | u;
    }
    if (!ok) { atomicOr(bad, 1); key = ~0ull; }
    keys[i] = key;
    idx[i] = (uint32_t)i;
}

__global__ void k_voxel_heads(const uint64_t *keys, int64_t n, int32_t *head) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    head[s] = (s == 0 || keys[s] != keys[s - 1]) ? 1 : 0;
}

__global__ void k_voxel_mean(const float *const *src, const uint64_t *keys, const uint32_t *idx, const int32_t *head,
                             const int32_t *vid, int64_t n, float *const *out, int64_t *count, const int32_t *bad) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s == n - 1) *count = *bad ? -1 : (int64_t)vid[s] + head[s];
    if (s >= n || !head[s]) return;
    int64_t e = s + 1;
    while (e < n && keys[e] == keys[s]) ++e;
    double sx = 0, sy = 0, sz = 0, snx = 0, sny = 0, snz = 0;
    for (int64_t t = s; t < e; ++t) {
        uint32_t i = idx[t];
        sx += src[0][i]; sy += src[1][i]; sz += src[2][i];
        snx += src[3][i]; sny += src[4][i]; snz += src[5][i];
    }
    double c = (double)(e - s);
    int64_t o = vid[s];
    out[0][o] = (float)(sx / c);
    out[1][o] = (float)(sy / c);
    out[2][o] = (float)(sz / c);
    // |sum n| without contraction, as a plain left-to-right evaluation
    double nn = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(snx, snx), __dmul_rn(sny, sny)), __dmul_rn(snz, snz)));
    if (nn > 0) {
        out[3][o] = (float)(snx / nn);
        out[4][o] = (float)(sny / nn);
        out[5][o] = (float)(snz / nn);
    } else {
        uint32_t i = idx[s];
        out[3][o] = src[3][i];
        out[4][o] = src[4][i];
        out[5][o] = src[5][i];
    }
}

size_t voxel_sort_bytes(int64_t n) {
    size_t bytes = 0;
    (void)rocprim::radix_sort_pairs(nullptr, bytes, (uint64_t *)nullptr, (uint64_t *)nullptr, (uint32_t *)nullptr,
                                    (uint32_t *)nullptr, (size_t)std::max<int64_t>(n, 1), 0, 63);
    return bytes;
}

// ws: keys (2n u64), idx (2n u32), head, vid (n i32 each), scan tmp, sort tmp; src/out: device arrays of 6 pointers
hipError_t launch_voxel(const float *const *src_dev, const float *const src[6], int64_t n, float v,
                        float *const *out_dev, int64_t *count, char *ws, size_t sort_bytes, hipStream_t s) {
    auto take = [&](size_t b) { char *r = ws; ws += (b + 255) & ~size_t(255); return r; };
    uint64_t *k0 = (uint64_t *)take(8 * n), *k1 = (uint64_t *)take(8 * n);
    uint32_t *i0 = (uint32_t *)take(4 * n), *i1 = (uint32_t *)take(4 * n);
    int32_t *head = (int32_t *)take(4 * n), *vid = (int32_t *)take(4 * n);
    int32_t *stmp = (int32_t *)take(4 * scan_tmp_elems(n));
    int32_t *bad = (int32_t *)take(256);
    void *sort_tmp = take(sort_bytes);
    hipError_t e;
    if ((e = fill<int32_t>(bad, 0, 1, s)) != hipSuccess) return e;
    unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_voxel_keys, dim3(nb), dim3(256), 0, s, src[0], src[1], src[2], n, (double)v, k0, i0, bad);
    size_t sb = sort_bytes;
    if ((e = rocprim::radix_sort_pairs(sort_tmp, sb, k0, k1, i0, i1, (size_t)n, 0, 63, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_voxel_heads, dim3(nb), dim3(256), 0, s, (const uint64_t *)k1, n, head);
    if ((e = exclusive_scan_i32(head, vid, n, stmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_voxel_mean, dim3(nb), dim3(256), 0, s, src_dev, (const uint64_t *)k1, (const uint32_t *)i1,
                       (const int32_t *)head, (const int32_t *)vid, n, out_dev, count, (const int32_t *)bad);
    return hipGetLastError();
}

size_t voxel_ws_bytes(int64_t n) {
    auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
    return 2 * r(8 * n) + 2 * r(4 * n) + 2 * r(4 * n) + r(4 * scan_tmp_elems(n)) + r(256) + r(voxel_sort_bytes(n)) +
           64 * 8;
}

}  // namespace lsr
