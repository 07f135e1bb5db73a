// 3-D grid index over every fragment of a batch (Sec. IV, eq. 1: cell index =
// (coordinate - origin) / cell length, taken with floor).  The cell edge is at
// least the search radius, so a radius query visits the 27 cells around the
// query's cell and finds the exact radius set.
//
// Build = bounding box -> grid shape -> counting sort of points by cell.  The
// sort is made deterministic by placing each point at its rank (by original
// index) inside its cell, so later floating-point sums see a fixed order.
#include "lsr_internal.h"

namespace lsr {

// ---------------------------------------------------------------- scan

constexpr int SCAN_T = 256, SCAN_V = 16, SCAN_B = SCAN_T * SCAN_V;

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + SCAN_B - 1) / SCAN_B) + 1; }

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive prefix of `v` across the block; returns the block total in *tot.
__device__ int32_t block_excl_scan(int32_t v, int32_t *sh, int32_t *tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k < nw; ++k) { int32_t t = sh[k]; sh[k] = run; run += t; }
        sh[nw] = run;
    }
    __syncthreads();
    int32_t r = sh[w] + inc - v;
    *tot = sh[nw];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_blocks(const int32_t *in, int32_t *out, int64_t n, int32_t *sums) {
    __shared__ int32_t sh[SCAN_T / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_V;
    int32_t v[SCAN_V];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_V; ++k) { v[k] = (base + k < n) ? in[base + k] : 0; s += v[k]; }
    int32_t tot;
    int32_t pre = block_excl_scan(s, sh, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_V; ++k) { if (base + k < n) out[base + k] = pre; pre += v[k]; }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int32_t *sums, int64_t nb) {
    __shared__ int32_t sh[1024 / 64 + 1];
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < nb ? sums[i] : 0;
        int32_t tot;
        int32_t pre = block_excl_scan(v, sh, &tot);
        if (i < nb) sums[i] = carry + pre;
        carry += tot;
    }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_add(int32_t *out, int64_t n, const int32_t *sums) {
    int64_t base = (int64_t)blockIdx.x * SCAN_B;
    int32_t add = sums[blockIdx.x];
    for (int k = threadIdx.x; k < SCAN_B; k += SCAN_T)
        if (base + k < n) out[base + k] += add;
}

hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_T), 0, s, out, n, (const int32_t *)tmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------- grid build

__global__ void __launch_bounds__(256) k_bbox(Frag *frag, const Blk *blk) {
    __shared__ uint32_t sh[6][4];
    const Blk b = blk[blockIdx.x];
    Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0, 0, 0};
    if (i < F.n) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { uint32_t o = f2ord(F.src[a][i]); mn[a] = o; mx[a] = o; }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], o, 64));
            mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], o, 64));
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) { sh[a][w] = mn[a]; sh[3 + a][w] = mx[a]; }
    __syncthreads();
    if (threadIdx.x < 3) {
        int a = threadIdx.x;
        uint32_t m0 = sh[a][0], m1 = sh[3 + a][0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { m0 = min(m0, sh[a][k]); m1 = max(m1, sh[3 + a][k]); }
        atomicMin(&F.bmin[a], m0);
        atomicMax(&F.bmax[a], m1);
    }
}

__global__ void k_bbox_init(Frag *frag, int nfrag) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfrag) return;
    for (int a = 0; a < 3; ++a) { frag[f].bmin[a] = 0xffffffffu; frag[f].bmax[a] = 0u; }
}

__global__ void k_grid_setup(Frag *frag, int nfrag, float r_cell) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfrag) return;
    Frag &F = frag[f];
    float mn[3], mx[3];
    bool finite = true;
    for (int a = 0; a < 3; ++a) {
        if (F.n > 0) { mn[a] = ord2f(F.bmin[a]); mx[a] = ord2f(F.bmax[a]); }
        else { mn[a] = 0.f; mx[a] = 0.f; }
        finite = finite && isfinite(mn[a]) && isfinite(mx[a]);
    }
    if (!finite) {                    // non-finite input: one cell holds every point (exact, slow)
        F.ox = F.oy = F.oz = 0.f;
        F.cell = 3.0e38f;
        F.gx = F.gy = F.gz = 1;
        return;
    }
    double ext[3] = {(double)mx[0] - mn[0], (double)mx[1] - mn[1], (double)mx[2] - mn[2]};
    double cell = fmax((double)r_cell * 1.001, 1e-6);
    const double cap = (double)F.cell_cap;
    for (int it = 0; it < 256; ++it) {
        double prod = (floor(ext[0] / cell) + 1) * (floor(ext[1] / cell) + 1) * (floor(ext[2] / cell) + 1);
        if (prod <= cap) break;
        cell *= fmax(1.01, 1.01 * cbrt(prod / cap));   // a coarser cell is still exact for the stencil
    }
    float fc = (float)cell;
    if ((double)fc < cell) fc = nextafterf(fc, 3.0e38f);
    F.ox = mn[0]; F.oy = mn[1]; F.oz = mn[2];
    F.cell = fc;
    F.gx = (int)(floor(ext[0] / (double)fc) + 1);
    F.gy = (int)(floor(ext[1] / (double)fc) + 1);
    F.gz = (int)(floor(ext[2] / (double)fc) + 1);
}

// Cell of each point and its arrival rank in the cell (the count's atomic
// return value; any order of arrival, since the rank fix below orders each
// cell by original index).
__global__ void __launch_bounds__(256) k_count(const Frag *frag, const Blk *blk, int32_t *cell_of_pt, int32_t *ccount,
                                               int32_t *arrival) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= F.n) return;
    int cx, cy, cz;
    cell_of(F, (double)F.src[0][i], (double)F.src[1][i], (double)F.src[2][i], cx, cy, cz);
    cx = min(max(cx, 0), F.gx - 1); cy = min(max(cy, 0), F.gy - 1); cz = min(max(cz, 0), F.gz - 1);
    int32_t gc = (int32_t)(F.cell_off + ((int64_t)cz * F.gy + cy) * F.gx + cx);
    cell_of_pt[F.off + i] = gc;
    arrival[F.off + i] = atomicAdd(&ccount[gc], 1);
}

__global__ void __launch_bounds__(256) k_scatter(const Frag *frag, const Blk *blk, const int32_t *cell_of_pt,
                                                 const int32_t *cstart, const int32_t *arrival, int32_t *tmp) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= F.n) return;
    int64_t g = F.off + i;
    tmp[cstart[cell_of_pt[g]] + arrival[g]] = (int32_t)g;
}

__global__ void __launch_bounds__(256) k_rankfix(const Frag *frag, const Blk *blk, const int32_t *cell_of_pt,
                                                 const int32_t *cstart, const int32_t *ccount, const int32_t *tmp,
                                                 float4 *sp, float *snx, float *sny, float *snz,
                                                 int32_t *sorig) {
    // One thread per sorted slot: the point the scatter parked in slot q (in
    // arrival order) moves to its final slot st + rank, rank = its order by
    // original index within the cell.  The writes stay inside the cell's slot
    // range; the point's own fields are gathered from the input.
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    const int q = b.start + threadIdx.x;
    if (q >= F.n) return;
    const int32_t g = tmp[F.off + q];
    const int i = (int)(g - F.off);
    int32_t gc = cell_of_pt[g];
    int32_t st = cstart[gc], cnt = ccount[gc], rank = 0;
    for (int32_t k = 0; k < cnt; ++k) rank += tmp[st + k] < g;
    int32_t d = st + rank;
    sp[d] = make_float4(F.src[0][i], F.src[1][i], F.src[2][i], 0.f);
    const bool has_n = F.src[3] && F.src[4] && F.src[5];       // stage calls may omit normals
    snx[d] = has_n ? F.src[3][i] : 0.f;
    sny[d] = has_n ? F.src[4][i] : 0.f;
    snz[d] = has_n ? F.src[5][i] : 0.f;
    sorig[d] = i;
}

hipError_t build_grids(GridBufs &g, float r_cell, hipStream_t s) {
    hipError_t e;
    if (g.ntot == 0) return hipSuccess;
    if ((e = fill<int32_t>(g.ccount, 0, g.ncells, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbox_init, dim3((g.nfrag + 63) / 64), dim3(64), 0, s, g.frag, g.nfrag);
    hipLaunchKernelGGL(k_bbox, dim3(g.nblk256), dim3(256), 0, s, g.frag, (const Blk *)g.blk256);
    hipLaunchKernelGGL(k_grid_setup, dim3((g.nfrag + 63) / 64), dim3(64), 0, s, g.frag, g.nfrag, r_cell);
    // arrival ranks in cursor[0, ntot) (ncells >= ntot), the scan's scratch from cursor + ncells
    hipLaunchKernelGGL(k_count, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       g.cell_of_pt, g.ccount, g.cursor);
    if ((e = exclusive_scan_i32(g.ccount, g.cstart, g.ncells, g.cursor + g.ncells, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)g.cell_of_pt, (const int32_t *)g.cstart, (const int32_t *)g.cursor, g.tmp);
    hipLaunchKernelGGL(k_rankfix, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)g.cell_of_pt, (const int32_t *)g.cstart, (const int32_t *)g.ccount,
                       (const int32_t *)g.tmp, g.sp, g.snx, g.sny, g.snz, g.sorig);
    return hipGetLastError();
}

}  // namespace lsr
