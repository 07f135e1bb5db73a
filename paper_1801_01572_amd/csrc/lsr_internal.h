// Internal declarations shared by the HIP translation units of liblsr.
//
// Data model.  A launch works on a batch of fragments (two per pair: P at
// 2b, Q at 2b+1).  Points of all fragments live in one internal index space
// [0, Ntot): fragment f owns [Frag::off, Frag::off + Frag::n).  Each stage is
// one kernel over the whole batch, so the launch count does not grow with the
// number of pairs.  A block of a per-point kernel never spans two fragments:
// the host builds a block table (fragment, first point) per block size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lsr.h"

namespace lsr {

constexpr int FD = 33;          // descriptor length: 3 features x 11 bins
constexpr int NB = 11;          // bins per feature
constexpr int SPR = 5;          // SPFH row in 16-byte units: 33 u16 bin counts, 5 zero u16, float scale (80 B)
constexpr int PK = 64;          // packed screen row: hi and lo bf16 halves, 32 each (30 dims + 2 slots)

struct Frag {
    const float *src[6];        // caller's SoA arrays for this fragment (already offset)
    int64_t off;                // first internal point index
    int32_t n;                  // points
    int32_t partner;            // the other fragment of the pair, or -1
    int64_t cell_off;           // first cell of this fragment's grid table
    int32_t cell_cap;           // cells reserved for the grid table
    int32_t pair;               // pair index, or -1
    int64_t pk_off;             // first packed screen row (rows padded to a multiple of 128)
    int32_t blk256_first;       // index of the fragment's first entry in the 256-point block table
    int32_t pad0;
    int64_t uoff;               // first point of the fragment in the caller's concatenated cloud
    // filled on the device by the grid kernels
    float ox, oy, oz, cell;     // grid origin (bounding-box minimum) and cell edge
    int32_t gx, gy, gz, pad;    // grid dimensions
    uint32_t bmin[3], bmax[3];  // bounding box, order-preserving integer encoding
};

struct Blk {                    // one entry of a block table
    int32_t frag;
    int32_t start;              // first point of the block, relative to the fragment
};

// Per-pair counters and scalars accumulated across stages.
struct PairState {
    unsigned long long n_valid[2];
    unsigned long long n_recip;
    unsigned long long n_consistent;
    unsigned long long n_inliers;
    unsigned long long sum_d2_fixed;   // inlier squared distances, fixed point
    unsigned long long n_fallback;
    unsigned long long trials_passed;
    unsigned long long scr_chunks;     // bf16 screen: (64-query group, 128-row chunk) visits of a full sweep
    unsigned long long scr_swept;      // ... visits made (centroid passes included)
    double T[16];
    double energy, mu_final;
    int32_t status, iters;
    int64_t k_off;                     // first consistent correspondence in the compact list
    int64_t c_off, c_cnt;              // the pair's reciprocal correspondences in the packed list
    float mean_desc[PK];               // centring vector of the bf16 screen (projected space)
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ double pdist2(double xi, double yi, double zi, double xj, double yj, double zj) {
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    return __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
}

// SplitMix64 (Steele, Lea and Flood 2014): the n-th output for a seed is the
// finaliser applied to the state seed + (n + 1) * golden-gamma.  Consecutive
// attempts of one draw slot only add the gamma to the state; the index draws
// use the upper 32 bits of the output.
constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

// 1/sqrt(x) and 1/x in double: the hardware estimate plus two Newton steps
// (relative error ~1e-16), a few instructions against the correctly rounded
// library sequences.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    double e = fma(-x * r, r, 1.0);
    r = fma(0.5 * r, e, r);
    e = fma(-x * r, r, 1.0);
    return fma(0.5 * r, e, r);
}
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ uint32_t splitmix64_hi(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

// First correspondence word of fragment f: words of 32 points, fragment
// ranges kept apart by one spare word per fragment.
__device__ __forceinline__ int64_t word_off(const Frag &F, int f) { return (F.off >> 5) + f; }

// Similar-polygon test of one edge (Algorithm 1's pre-rejection): packed
// correspondences (p.xyz, q.x), (q.y, q.z, ...) of the edge's two ends; the
// squared lengths in P and in Q must each be at least tau^2 times the other
// (FP64 on the float inputs, pinned fma order); a zero edge fails.
__device__ __forceinline__ bool edge_ok(const float4 &a0, const float4 &a1, const float4 &b0, const float4 &b1,
                                        double t2) {
    double a = pdist2(a0.x, a0.y, a0.z, b0.x, b0.y, b0.z);
    double c = pdist2(a0.w, a1.x, a1.y, b0.w, b1.x, b1.y);
    return !(a == 0.0 || c == 0.0 || a < t2 * c || c < t2 * a);
}

// XCD-aware block order.  The device hands workgroups to its 8 XCDs
// round-robin (workgroup w runs on XCD w % 8), so consecutive entries of a
// block table (neighbouring points, or one fragment's blocks) would run on
// different XCDs and each XCD's L2 would fetch the data they share.
// Workgroup w takes table entry (w % 8) per + w / 8 instead: each XCD walks a
// contiguous eighth of the table.  The grid has xcd_grid(nblk) = 8 per
// workgroups, per = ceil(nblk / 8); entries >= nblk do nothing.
__device__ __forceinline__ int xcd_block(int nblk) {
    const int per = (nblk + 7) >> 3;
    return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}
static inline int xcd_grid(int nblk) { return 8 * ((nblk + 7) / 8); }

__device__ __forceinline__ uint32_t f2ord(float f) {   // order-preserving float -> uint
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __host__ __forceinline__ float ord2f(uint32_t u) {
    uint32_t v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
#ifdef __HIP_DEVICE_COMPILE__
    return __uint_as_float(v);
#else
    float f; __builtin_memcpy(&f, &v, 4); return f;
#endif
}

// Cell coordinates of a point in a fragment's grid (double precision keeps
// |cell(a) - cell(b)| <= 1 whenever |a - b| <= r < cell).
__device__ __forceinline__ void cell_of(const Frag &F, double x, double y, double z, int &cx, int &cy, int &cz) {
    double c = (double)F.cell;
    cx = (int)floor((x - (double)F.ox) / c);
    cy = (int)floor((y - (double)F.oy) / c);
    cz = (int)floor((z - (double)F.oz) / c);
}

// ---------------------------------------------------------------- workspace views

struct GridBufs {              // built per batch by build_grids()
    Frag *frag;                // device, nfrag
    int nfrag;
    int64_t ntot;              // total points
    int64_t ncells;            // total cells
    int32_t *cell_of_pt;       // internal index -> linear cell (within fragment table)
    int32_t *cstart;           // ncells + 1: global sorted position of each cell
    int32_t *ccount;           // ncells
    int32_t *cursor;           // ncells (>= ntot) + scan scratch: each point's arrival rank in its cell
    int32_t *tmp;              // ntot, unstable scatter
    float4 *sp;                // sorted coordinates (x, y, z, 0): one 16-byte load per candidate
    float *snx, *sny, *snz;    // sorted input normals
    int32_t *sorig;            // sorted position -> original index within the fragment
    Blk *blk256; int nblk256;  // block tables: 256 points per block
    Blk *blk512; int nblk512;  // 512 points per block
    int64_t *frag_off;         // nfrag + 1 internal offsets (device)
    int64_t pk_rows;           // packed screen rows (each fragment padded to a multiple of 128)
    int32_t max_np;            // largest P fragment of the batch (host copy)
};

struct DescBufs {
    double *nx, *ny, *nz;      // estimated normals, sorted order
    uint4 *spfh;               // sorted order, ntot x SPR: bin counts (u16) and the scale 1/kp (last word)
    int32_t *knb;              // neighbour count within r_feature, sorted order
    float *F;                  // descriptors, original order (fragment-relative via Frag::off), ntot x 33
    int32_t *valid;            // original order
    uint16_t *pk;              // bf16 packed screen rows (hi | lo), padded per fragment, pk_rows x 64
};

struct MatchBufs {
    int32_t *nn;               // original order: nearest neighbour (index in partner fragment)
    unsigned long long *nnkey; // float32 scan split over candidate ranges: (distance bits, index) minima
    float *dist;
    uint8_t *mutual;           // original order
    float4 *cpack;             // reciprocal correspondences packed per pair: (px, py, pz, qx), (qy, qz, i, 0)
    uint2 *cwords;             // per 32 P points: bits of those with a correspondence, packed position of the first
    int32_t *flag;             // consistency flags, original order (int32 for the scan)
    int32_t *kpos;             // exclusive scan of flags over the batch
    float *kp, *kq;            // consistent correspondences, compacted: xyz of p and q (3 floats each)
    int32_t *ki;               // compacted P index of each consistent correspondence
};

struct RansacBufs {            // one pair's RANSAC hypotheses (capacity cap)
    unsigned long long *ctr;   // [0] survivors appended, [1] fitted, [2] largest completed inlier count
    int4 *pos;                 // packed correspondence positions of the four members
    int32_t *t;                // hypothesis index
    double *T;                 // fitted [R | t], 12 per survivor
    int32_t *cnt;              // inliers; -1: no unique fit; -2: stopped, cannot be chosen
    double *ss;                // sum of the inliers' squared nearest distances
    int64_t cap;
};

struct TrialBlk {              // consistency trials handled by one block
    int32_t pair;
    int32_t pad;
    int64_t first;             // first trial index of the block
    int64_t count;             // trials of this pair (all blocks)
};

struct SurfelWs {              // scratch of one surfel correction (surfel_carve)
    float *tmp;                // 6 x n updates at the surfels' own indices
    int32_t *keep, *pos;       // keep flags and their exclusive scan
    int32_t *scan_tmp;
    double *T_old, *T_new;     // keyframe table: n_kf x 16 each
    int32_t *t_kf;
    float **out_ptrs;          // the six output array pointers (device copy)
};

// ---------------------------------------------------------------- launchers

hipError_t build_grids(GridBufs &g, float r_cell, hipStream_t s);
hipError_t launch_normals(const GridBufs &g, float r_normal, DescBufs &d, double *nrm_orig, hipStream_t s);
hipError_t launch_normals_inject(const GridBufs &g, const double *nrm_orig, DescBufs &d, hipStream_t s);
hipError_t launch_spfh(const GridBufs &g, float r_feature, DescBufs &d, hipStream_t s);
hipError_t launch_spfh_out(const GridBufs &g, const DescBufs &d, float *out, int32_t *kout, hipStream_t s);
hipError_t launch_fpfh(const GridBufs &g, float r_feature, DescBufs &d, PairState *ps, hipStream_t s);
hipError_t launch_mutual(const GridBufs &g, MatchBufs &m, PairState *ps, hipStream_t s);
hipError_t launch_consistency(const GridBufs &g, MatchBufs &m, PairState *ps, const TrialBlk *tb, int ntb,
                              float tau, uint64_t seed, int shape, int32_t *scan_tmp, hipStream_t s);
size_t corr_words(int64_t ntot, int nfrag);
// Packs the correspondences of every P point (reciprocal ones, or every valid
// descriptor neighbour when one_way) in ascending P index into m.cpack, the
// per-32-point words into m.cwords, and each pair's list into ps (c_off,
// c_cnt).  Uses m.flag and m.kpos as scratch.
hipError_t launch_corr_pack(const GridBufs &g, MatchBufs &m, PairState *ps, bool one_way, int32_t *scan_tmp,
                            hipStream_t s);
hipError_t launch_compact(const GridBufs &g, MatchBufs &m, PairState *ps, int32_t *scan_tmp, hipStream_t s);
size_t ransac_bytes(int64_t cap);
RansacBufs ransac_carve(void *mem, int64_t cap);
hipError_t launch_ransac(const GridBufs &g, const DescBufs &d, MatchBufs &m, PairState *ps, RansacBufs R,
                         int64_t n_hyp, const lsr_params &prm, int32_t *scan_tmp, lsr_ransac_result *out,
                         const lsr_ransac_trace *tr, hipStream_t s);
hipError_t launch_gnc(const GridBufs &g, const MatchBufs &m, PairState *ps, int npairs, const lsr_params &prm,
                      hipStream_t s);
hipError_t launch_gnc_direct(const double *p, const double *q, int64_t m, const lsr_params &prm, PairState *ps,
                             hipStream_t s);
hipError_t launch_verify(const GridBufs &g, const DescBufs &d, PairState *ps, float delta, int normal_check,
                         float normal_cos, hipStream_t s);
hipError_t launch_finalize(const GridBufs &g, PairState *ps, int npairs, const lsr_params &prm, lsr_result *out,
                           hipStream_t s);
hipError_t launch_align_loss(const float *const P[3], const float *const Q[3], const int32_t *corr,
                             const int32_t *corr_prob, int64_t m_tot, const double *T, const double *mu,
                             const double *dE, double *partial, int64_t nblocks, const int64_t *blk_first,
                             const int32_t *blk_prob_first, int nprob, double *E_out, float *const dP[3],
                             float *const dQ[3], double *dxi, hipStream_t s);

size_t surfel_ws_bytes(int64_t n, int32_t n_kf);
SurfelWs surfel_carve(char *ws, int64_t n, int32_t n_kf);
hipError_t launch_surfel_correct(const float *const src[6], const int32_t *t0, const int32_t *tu, int64_t n,
                                 const SurfelWs &w, int32_t n_kf, const lsr_camera &cam, float *const *out_dev,
                                 int32_t *new_index, int32_t *k_obs, int64_t *n_kept, hipStream_t s);

hipError_t launch_edge_info(const GridBufs &g, const double *A, int n_edges, float eps, double *partial,
                            double *info, int64_t *count, hipStream_t s);
size_t loop_scratch_bytes(int n, int n_loops);
hipError_t launch_loop_solve(int n, const double *T_init, const lsr_edge *odo, const double *L_odo,
                             const lsr_edge *loops, int n_loops, const double *L_loop, const int64_t *cnt_loop,
                             const lsr_loop_params &prm, double *scratch, double *T_out, lsr_loop_result *res,
                             hipStream_t s);

// Optional stage timing: when enabled, launchers record an event after each
// named step on the launch stream (eager runs only, never under capture).
void tmark(const char *name, hipStream_t s);

// device scans
hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
template <typename T>
inline hipError_t fill(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)nb), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

template <typename T>
__global__ void k_copy(T *dst, const T *src, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}
template <typename T>
inline hipError_t copy(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)nb), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace lsr
