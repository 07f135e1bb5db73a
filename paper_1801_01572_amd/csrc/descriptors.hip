// Per-point geometry on the grid: normals, SPFH and FPFH.
//
// Normals: principal component analysis of the radius-r_normal neighbourhood
// plus the point (normal estimation radius of Sec. IV), FP64, oriented by
// the input normal; fewer than 3 points keep the normalised input normal.
//
// FPFH (the descriptor of Algorithm 1; definition from the cited FPFH work):
// for each neighbour pair, a Darboux frame u = n_s, v = u x e / |u x e|,
// w = u x v, with the source s the endpoint whose normal makes the smaller
// angle with the line towards the other; features alpha = v.n_t,
// phi = u.e, theta = atan2(w.n_t, u.n_t) binned into 11 bins each.  SPFH_i is
// the histogram divided by the number of non-degenerate pairs;
// FPFH_i = SPFH_i + (1/k_i) sum_j SPFH_j / |p_j - p_i|, each 11-bin block then
// scaled to unit sum.  Pair features are computed in FP64 so that bin and
// source decisions agree with an FP64 evaluation except within rounding of a
// boundary.
#include <cmath>

#include "lsr_internal.h"

namespace lsr {

struct GridView {
    const int32_t *cstart, *ccount;
    const float4 *p;           // sorted (x, y, z, 0)
};

// Visit every sorted point within the 27-cell stencil of (px, py, pz): the
// three cells adjacent along x are consecutive in the table, so the stencil is
// nine contiguous runs of the sorted arrays.  For a search radius r of at most
// half a cell (r >= 0 given) a point within r of p lies, along each axis, in
// p's cell and the neighbour on the side of p's half of the cell: 2 x 2 x 2
// cells, four runs.
template <class Fn>
__device__ __forceinline__ void for_stencil(const Frag &F, const GridView &g, double px, double py, double pz, Fn &&fn,
                                            double r = -1.0) {
    const double c = (double)F.cell;
    const double fx = (px - (double)F.ox) / c, fy = (py - (double)F.oy) / c, fz = (pz - (double)F.oz) / c;
    const int cx = (int)floor(fx), cy = (int)floor(fy), cz = (int)floor(fz);
    int lx = cx - 1, ly = cy - 1, lz = cz - 1, hx = cx + 1, hy = cy + 1, hz = cz + 1;
    if (r >= 0.0 && r <= 0.499999 * c) {
        lx = fx - cx < 0.5 ? cx - 1 : cx; hx = lx + 1;
        ly = fy - cy < 0.5 ? cy - 1 : cy; hy = ly + 1;
        lz = fz - cz < 0.5 ? cz - 1 : cz; hz = lz + 1;
    }
    int x0 = max(lx, 0), x1 = min(hx, F.gx - 1);
    if (x0 > x1) return;
    for (int z = max(lz, 0); z <= min(hz, F.gz - 1); ++z) {
        for (int y = max(ly, 0); y <= min(hy, F.gy - 1); ++y) {
            int64_t row = F.cell_off + ((int64_t)z * F.gy + y) * F.gx;
            int32_t b = g.cstart[row + x0];
            int32_t e = g.cstart[row + x1] + g.ccount[row + x1];
            for (int32_t k = b; k < e; ++k) fn(k);
        }
    }
}

// ---------------------------------------------------------------- normals

// Smallest-eigenvalue eigenvector of a symmetric 3x3 matrix by cyclic Jacobi
// rotations (each rotation zeroes one off-diagonal entry).
__device__ void jacobi_min_vec(double a00, double a01, double a02, double a11, double a12, double a22, double v[3]) {
    double A[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 32; ++sweep) {
        double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        double diag = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off == 0.0 || off <= 1e-18 * diag) break;
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            double apq = A[p][q];
            if (apq == 0.0) continue;
            double th = (A[q][q] - A[p][p]) / (2.0 * apq);
            double t = fabs(th) > 1e150 ? 0.5 / th : copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double kp = A[k][p], kq = A[k][q];
                A[k][p] = c * kp - s * kq;
                A[k][q] = s * kp + c * kq;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double pk = A[p][k], qk = A[q][k];
                A[p][k] = c * pk - s * qk;
                A[q][k] = s * pk + c * qk;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double kp = V[k][p], kq = V[k][q];
                V[k][p] = c * kp - s * kq;
                V[k][q] = s * kp + c * kq;
            }
        }
    }
    int m = 0;
    if (A[1][1] < A[m][m]) m = 1;
    if (A[2][2] < A[m][m]) m = 2;
    double x = m == 0 ? V[0][0] : (m == 1 ? V[0][1] : V[0][2]);
    double y = m == 0 ? V[1][0] : (m == 1 ? V[1][1] : V[1][2]);
    double z = m == 0 ? V[2][0] : (m == 1 ? V[2][1] : V[2][2]);
    double inv = 1.0 / sqrt(x * x + y * y + z * z);
    v[0] = x * inv; v[1] = y * inv; v[2] = z * inv;
}

__global__ void __launch_bounds__(256) k_normals(const Frag *frag, const Blk *blk, int nblk, GridView g,
                                                 const float *snx, const float *sny, const float *snz,
                                                 const int32_t *sorig, double r2, double *nx, double *ny, double *nz,
                                                 double *nrm_orig) {
    const int bi = xcd_block(nblk);                   // neighbouring blocks share candidates
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= F.n) return;
    int64_t s = F.off + i;
    const float4 p4 = g.p[s];
    double px = p4.x, py = p4.y, pz = p4.z;
    // shifted sums (origin at p_i): sum d, sum d d^T
    double m = 1, s1x = 0, s1y = 0, s1z = 0, sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
    const double rn = sqrt(r2);
    for_stencil(F, g, px, py, pz, [&](int32_t k) {
        const float4 q4 = g.p[k];
        double qx = q4.x, qy = q4.y, qz = q4.z;
        double d2 = pdist2(px, py, pz, qx, qy, qz);
        if (d2 > 0.0 && d2 <= r2) {
            double dx = qx - px, dy = qy - py, dz = qz - pz;
            m += 1; s1x += dx; s1y += dy; s1z += dz;
            sxx += dx * dx; sxy += dx * dy; sxz += dx * dz; syy += dy * dy; syz += dy * dz; szz += dz * dz;
        }
    }, rn);
    double ix = snx[s], iy = sny[s], iz = snz[s];
    double v[3];
    if (m < 3) {
        double l = sqrt(ix * ix + iy * iy + iz * iz);
        double inv = l > 0 ? 1.0 / l : 0.0;
        v[0] = ix * inv; v[1] = iy * inv; v[2] = iz * inv;
    } else {
        double im = 1.0 / m;
        double mx = s1x * im, my = s1y * im, mz = s1z * im;
        jacobi_min_vec(sxx * im - mx * mx, sxy * im - mx * my, sxz * im - mx * mz,
                       syy * im - my * my, syz * im - my * mz, szz * im - mz * mz, v);
        if (v[0] * ix + v[1] * iy + v[2] * iz < 0) { v[0] = -v[0]; v[1] = -v[1]; v[2] = -v[2]; }
    }
    nx[s] = v[0]; ny[s] = v[1]; nz[s] = v[2];
    if (nrm_orig) {
        int64_t o = (F.off + sorig[s]) * 3;
        nrm_orig[o] = v[0]; nrm_orig[o + 1] = v[1]; nrm_orig[o + 2] = v[2];
    }
}

hipError_t launch_normals(const GridBufs &g, float r_normal, DescBufs &d, double *nrm_orig, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    GridView gv{g.cstart, g.ccount, g.sp};
    double r2 = (double)r_normal * (double)r_normal;
    hipLaunchKernelGGL(k_normals, dim3(xcd_grid(g.nblk256)), dim3(256), 0, s, (const Frag *)g.frag,
                       (const Blk *)g.blk256, g.nblk256, gv,
                       (const float *)g.snx, (const float *)g.sny, (const float *)g.snz, (const int32_t *)g.sorig,
                       r2, d.nx, d.ny, d.nz, nrm_orig);
    return hipGetLastError();
}

// Normals given by the caller (original order, n x 3) copied into sorted order.
__global__ void __launch_bounds__(256) k_normals_inject(const Frag *frag, const Blk *blk, const int32_t *sorig,
                                                        const double *nrm_orig, double *nx, double *ny, double *nz) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= F.n) return;
    int64_t s = F.off + i;
    int64_t o = (F.off + sorig[s]) * 3;
    nx[s] = nrm_orig[o]; ny[s] = nrm_orig[o + 1]; nz[s] = nrm_orig[o + 2];
}

hipError_t launch_normals_inject(const GridBufs &g, const double *nrm_orig, DescBufs &d, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_normals_inject, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)g.sorig, nrm_orig, d.nx, d.ny, d.nz);
    return hipGetLastError();
}

// ---------------------------------------------------------------- SPFH

// rsqrt_nr, rcp_nr (lsr_internal.h): relative error ~1e-16, far inside the
// bin-decision margins.

// theta's bin edges theta_k = -pi + 2 pi k / 11 as values of the pseudo-angle
// pa(x, y) = 1 - x / (|x| + |y|) for y >= +0 and x / (|x| + |y|) - 1 for y < 0
// (sign bit), which increases with atan2(y, x) on (-pi, pi].
struct ThetaEdges { double e[NB - 1]; };

__device__ __forceinline__ int bin11(double x) {       // x in bin units
    double f = floor(x);
    f = fmin(fmax(f, 0.0), (double)(NB - 1));
    return (int)f;
}

constexpr int SPFH_T = 256;

// For each neighbour pair the Darboux frame u = n_s, v = (u x e)/|u x e|,
// w = u x v with the source the endpoint whose normal makes the smaller angle
// with the connecting line (n_i.e >= -(n_j.e): source i).  With the
// unnormalised line d = p_j - p_i every feature follows without dividing by
// |d| more than once: the source test is (n_i + n_j).d >= 0; with
// c = u x d_s and l2 = |c|^2: alpha = (c.n_t) / sqrt(l2), phi = (u.d_s)/|d|,
// theta = atan2(w.n_t, u.n_t) with w.n_t = ((u.d_s)(u.n_t) - (d_s.n_t)(u.u)) / sqrt(l2).
// Returns false for a degenerate frame (|u x e| <= 1e-12: the pair is skipped).
__device__ __forceinline__ bool pair_bins(double px, double py, double pz, double ax, double ay, double az,
                                          const float4 q4, double bx, double by, double bz, const ThetaEdges &te,
                                          int &b0, int &b1, int &b2) {
    double dx = (double)q4.x - px, dy = (double)q4.y - py, dz = (double)q4.z - pz;
    double d2 = __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
    bool src_i = (ax + bx) * dx + (ay + by) * dy + (az + bz) * dz >= 0.0;
    double ux = src_i ? ax : bx, uy = src_i ? ay : by, uz = src_i ? az : bz;
    double tx = src_i ? bx : ax, ty = src_i ? by : ay, tz = src_i ? bz : az;
    if (!src_i) { dx = -dx; dy = -dy; dz = -dz; }
    double cx = uy * dz - uz * dy, cy = uz * dx - ux * dz, cz = ux * dy - uy * dx;
    double l2 = cx * cx + cy * cy + cz * cz;
    if (!(l2 > 1e-24 * d2)) return false;
    double il = rsqrt_nr(l2);
    double ud = ux * dx + uy * dy + uz * dz;
    double ut = ux * tx + uy * ty + uz * tz;
    double dt = dx * tx + dy * ty + dz * tz;
    double uu = ux * ux + uy * uy + uz * uz;
    double alpha = (cx * tx + cy * ty + cz * tz) * il;
    double phi = ud * rsqrt_nr(d2);
    double wt = (ud * ut - dt * uu) * il;             // w . n_t
    double sa = fabs(ut) + fabs(wt);
    double pa = 0.0;
    if (sa > 0.0) {
        double q = ut * rcp_nr(sa);
        pa = signbit(wt) ? q - 1.0 : 1.0 - q;
    }
    int bt = 0;
#pragma unroll
    for (int e = 0; e < NB - 1; ++e) bt += pa >= te.e[e];
    b0 = bin11(NB * (alpha + 1.0) / 2.0);
    b1 = NB + bin11(NB * (phi + 1.0) / 2.0);
    b2 = 2 * NB + bt;
    return true;
}

constexpr int SPFH_RING = 128;   // per-wavefront ring of (owner lane, neighbour) pairs

__device__ __forceinline__ uint32_t lanes_below64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wavefront's 64 points are taken 16 at a time, as in the FPFH kernel: the
// group's points that share a grid row find all their neighbours in nine
// x-runs, and each step tests 4 candidates against the 16 points (lane
// (i, k) = (l % 16, l / 16) tests point i against candidate c0 + k, with the
// same FP64 distance as the per-point stencil).  Every lane runs every step,
// so the loop is uniform and the ring of found pairs (owner, j) keeps its
// cursors in scalar registers.  Whenever 64 pairs are parked each lane bins
// one (FP64 Darboux frame, hardware rsq/rcp seeds with two Newton steps,
// theta by pseudo-angle comparisons against edges precomputed on the host);
// bins are counted with integer LDS atomics into the owner's histogram (order
// independent).  kp is the sum of the alpha block (each counted pair adds one
// to every block).
__global__ void __launch_bounds__(SPFH_T) k_spfh(const Frag *frag, const Blk *blk, int nblk, GridView g,
                                                 const double *nxa, const double *nya, const double *nza, double r2,
                                                 ThetaEdges te, uint4 *spfh, int32_t *knb) {
    __shared__ uint32_t hist[SPFH_T * FD];
    __shared__ int2 ring_all[SPFH_T / 64][SPFH_RING];
    // XCD-aware order: neighbouring blocks share most candidate rows
    const int bi = xcd_block(nblk);
    if (bi >= nblk) return;
    uint32_t *h = hist + threadIdx.x * FD;
#pragma unroll
    for (int c = 0; c < FD; ++c) h[c] = 0;
    const Blk b = blk[bi];
    const Frag &F = frag[b.frag];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pi = lane & 15, kk = lane >> 4;
    int2 *ring = ring_all[wv];
    uint32_t *hw = hist + wv * 64 * FD;               // this wavefront's 64 histograms
    const int64_t s0 = F.off + b.start + wv * 64;      // sorted index of the wavefront's first point
    const int i = b.start + threadIdx.x;
    const bool live = i < F.n;
    const int64_t s = F.off + i;
    // bin the pair parked in slot e (owner o = point index in the wavefront, neighbour j)
    auto bin_pair = [&](int2 e) {
        const int64_t so = s0 + e.x;
        const float4 o4 = g.p[so];
        int b0, b1, b2;
        if (pair_bins(o4.x, o4.y, o4.z, nxa[so], nya[so], nza[so], g.p[e.y], nxa[e.y], nya[e.y], nza[e.y], te, b0, b1,
                      b2)) {
            uint32_t *ho = hw + e.x * FD;
            atomicAdd(ho + b0, 1u);
            atomicAdd(ho + b1, 1u);
            atomicAdd(ho + b2, 1u);
        }
    };
    wave_sync_lds();
    const double c = (double)F.cell;
    uint32_t head = 0, tail = 0;                      // ring cursors (uniform)
    int kmine = 0;                                    // neighbour count of this lane's own point
    for (int gq = 0; gq < 4; ++gq) {
        const int gbase = b.start + wv * 64 + gq * 16;
        if (gbase >= F.n) break;                      // uniform
        const int ip = gbase + pi;
        const bool pl = ip < F.n;
        const float4 p4 = pl ? g.p[F.off + ip] : make_float4(0.f, 0.f, 0.f, 0.f);
        const double px = p4.x, py = p4.y, pz = p4.z;
        const int cx = (int)floor((px - (double)F.ox) / c), cy = (int)floor((py - (double)F.oy) / c),
                  cz = (int)floor((pz - (double)F.oz) / c);
        const int x0i = max(cx - 1, 0), x1i = min(cx + 1, F.gx - 1);
        int kc = 0;
        uint64_t pend = __ballot(pl && kk == 0);
        while (pend) {
            const int lead = __builtin_ctzll(pend);
            const int ry = __builtin_amdgcn_readlane(cy, lead), rz = __builtin_amdgcn_readlane(cz, lead);
            const bool inrow = pl && ((pend >> pi) & 1) && cy == ry && cz == rz;
            pend &= ~__ballot(inrow && kk == 0);
            const bool use = inrow && x0i <= x1i;
            int x0 = use ? x0i : INT_MAX, x1 = use ? x1i : INT_MIN;
            for (int o = 1; o < 16; o <<= 1) {
                x0 = min(x0, __shfl_xor(x0, o, 64));
                x1 = max(x1, __shfl_xor(x1, o, 64));
            }
            x0 = __builtin_amdgcn_readfirstlane(x0);
            x1 = __builtin_amdgcn_readfirstlane(x1);
            if (x0 > x1) continue;
            for (int z = max(rz - 1, 0); z <= min(rz + 1, F.gz - 1); ++z) {
                for (int y = max(ry - 1, 0); y <= min(ry + 1, F.gy - 1); ++y) {
                    const int64_t row = F.cell_off + ((int64_t)z * F.gy + y) * F.gx;
                    const int32_t rb = g.cstart[row + x0], re = g.cstart[row + x1] + g.ccount[row + x1];
                    // four steps per iteration, their candidate loads issued together
                    // (a lane past the run's end reads the run's last candidate)
                    auto test = [&](int32_t j, const float4 &q4) {
                        const double d2 = pdist2(px, py, pz, (double)q4.x, (double)q4.y, (double)q4.z);
                        const bool hit = j < re && inrow && d2 > 0.0 && d2 <= r2;
                        kc += hit ? 1 : 0;
                        const uint64_t m = __ballot(hit);
                        if (hit) ring[(tail + lanes_below64(m)) & (SPFH_RING - 1)] = make_int2(gq * 16 + pi, j);
                        tail += __popcll(m);
                        if (tail - head >= 64) {      // every lane bins one parked pair
                            wave_sync_lds();
                            bin_pair(ring[(head + lane) & (SPFH_RING - 1)]);
                            head += 64;
                            wave_sync_lds();
                        }
                    };
                    for (int32_t c0 = rb; c0 < re; c0 += 16) {
                        const int32_t j0 = c0 + kk, j1 = j0 + 4, j2 = j0 + 8, j3 = j0 + 12;
                        const float4 q0 = g.p[min(j0, re - 1)], q1 = g.p[min(j1, re - 1)];
                        const float4 q2 = g.p[min(j2, re - 1)], q3 = g.p[min(j3, re - 1)];
                        test(j0, q0);
                        if (c0 + 4 < re) test(j1, q1);  // uniform
                        if (c0 + 8 < re) test(j2, q2);
                        if (c0 + 12 < re) test(j3, q3);
                    }
                }
            }
        }
        // neighbour count of point gq * 16 + pi: the four lanes that tested it
        kc += __shfl_xor(kc, 16, 64);
        kc += __shfl_xor(kc, 32, 64);
        const int kg = __shfl(kc, lane & 15, 64);
        if (kk == gq) kmine = kg;
    }
    // drain with the whole wavefront
    wave_sync_lds();
    while (head != tail) {
        const uint32_t n = min(64u, tail - head);
        if ((uint32_t)lane < n) bin_pair(ring[(head + lane) & (SPFH_RING - 1)]);
        head += n;
    }
    wave_sync_lds();
    const int k = kmine;
    if (!live) return;
    uint32_t kp = 0;
#pragma unroll
    for (int c = 0; c < NB; ++c) kp += h[c];
    // SPFH_i = counts / kp, stored as the exact counts (u16) and 1/kp.  Beyond
    // 65535 pairs the counts are rescaled to 16 bits (relative error <= 2^-16).
    float sc = kp > 0 ? 1.0f / (float)kp : 0.0f;
    uint32_t w[4 * SPR];
#pragma unroll
    for (int m = 0; m < 4 * SPR; ++m) w[m] = 0u;
    uint32_t hc[FD];
#pragma unroll
    for (int c = 0; c < FD; ++c) hc[c] = h[c];
    if (kp > 65535) {
#pragma unroll
        for (int c = 0; c < FD; ++c) hc[c] = (uint32_t)((double)hc[c] * (65535.0 / (double)kp) + 0.5);
        sc = 1.0f / 65535.0f;
    }
#pragma unroll
    for (int c = 0; c < FD; ++c) w[c >> 1] |= (hc[c] & 0xffffu) << (16 * (c & 1));
    w[4 * SPR - 1] = __float_as_uint(sc);
    uint4 *o = spfh + s * SPR;
#pragma unroll
    for (int q = 0; q < SPR; ++q) o[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    knb[s] = k;
}

hipError_t launch_spfh(const GridBufs &g, float r_feature, DescBufs &d, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    GridView gv{g.cstart, g.ccount, g.sp};
    double r2 = (double)r_feature * (double)r_feature;
    ThetaEdges te;
    const double PI = 3.14159265358979323846;
    for (int k = 1; k < NB; ++k) {
        double t = -PI + 2.0 * PI * k / NB, x = std::cos(t), y = std::sin(t), sa = std::fabs(x) + std::fabs(y);
        te.e[k - 1] = std::signbit(y) ? x / sa - 1.0 : 1.0 - x / sa;
    }
    hipLaunchKernelGGL(k_spfh, dim3(xcd_grid(g.nblk256)), dim3(SPFH_T), 0, s, (const Frag *)g.frag,
                       (const Blk *)g.blk256, g.nblk256, gv,
                       (const double *)d.nx, (const double *)d.ny, (const double *)d.nz, r2, te, d.spfh, d.knb);
    return hipGetLastError();
}

// SPFH and neighbour count in original order (stage output).
__global__ void __launch_bounds__(256) k_spfh_out(const Frag *frag, const Blk *blk, const int32_t *sorig,
                                                  const uint4 *spfh, const int32_t *knb, float *out, int32_t *kout) {
    const Blk b = blk[blockIdx.x];
    const Frag &F = frag[b.frag];
    int i = b.start + threadIdx.x;
    if (i >= F.n) return;
    int64_t s = F.off + i, o = F.off + sorig[s];
    const uint32_t *w = (const uint32_t *)(spfh + s * SPR);
    const float sc = __uint_as_float(w[4 * SPR - 1]);
    for (int c = 0; c < FD; ++c) out[o * FD + c] = (float)((w[c >> 1] >> (16 * (c & 1))) & 0xffffu) * sc;
    kout[o] = knb[s];
}

hipError_t launch_spfh_out(const GridBufs &g, const DescBufs &d, float *out, int32_t *kout, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spfh_out, dim3(g.nblk256), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       (const int32_t *)g.sorig, (const uint4 *)d.spfh, (const int32_t *)d.knb, out, kout);
    return hipGetLastError();
}

// ---------------------------------------------------------------- FPFH

typedef float f32x4v __attribute__((ext_vector_type(4)));

// The neighbour sum of FPFH_i is a sparse product: sum_j w_ij C_j with
// w_ij = scale_j / |p_j - p_i| over the r_f neighbours j and C_j the 33
// integer counts of SPFH_j (SPFH_j = scale_j C_j).  A wavefront takes 16
// consecutive sorted points at a time.  Sorted order is cell order with x
// fastest, so the group's points that share a grid row (cy, cz) are
// contiguous, ordered by cx, and all their neighbours lie in nine x-runs:
// rows (cy + dy, cz + dz), cells [first cx - 1, last cx + 1].  Each step
// covers 4 candidates of a run: lane (i, k) = (l % 16, l / 16) forms w for
// point i and candidate j = c0 + k (0 unless j is within r_f of p_i, the
// same FP64 test as the per-point stencil) and loads the counts of j for bins
// 2i and 2i + 1 (one word of the row) and the row's last 16 bytes (bin 32, its
// zero pad, the scale); three 16x16x4 f32 MFMAs add W (16 x 4) times C (4 x 48)
// into the group's sums, the even bins in the first, the odd in the second.  A group spanning several rows takes one pass per
// row, each with W masked to that row's points.  Only the float32 summation
// order differs from a per-point loop.  Seven wavefronts per SIMD (72 VGPRs,
// 24 bytes of spills; four at the unconstrained 104) hide more of the
// candidate-row gathers: 18.4 -> 17.4 ms at five, 17.1 -> 16.5 ms at six,
// 16.2 ms at seven, on 256 pairs of 50k-point fragments.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_fpfh(const Frag *frag, const Blk *blk, int nblk, GridView g,
                                              const int32_t *sorig, const uint4 *spfh, const int32_t *knb, double r2,
                                              float *Fout, int32_t *valid, PairState *ps) {
    __shared__ float red[4][16][49];                  // per wavefront: 16 points x 48 bins (+1 pad)
    __shared__ int cnt[4];
    // XCD-aware order: neighbouring blocks share most candidate rows
    const int bi = xcd_block(nblk);
    if (bi >= nblk) return;
    const Blk b = blk[bi];
    const Frag &F = frag[b.frag];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pi = lane & 15, kk = lane >> 4;
    const double c = (double)F.cell;
    const f32x4v zero = {0.f, 0.f, 0.f, 0.f};
    int nok = 0;                                      // valid descriptors written by this lane
    for (int gq = 0; gq < 4; ++gq) {
        const int base = b.start + wv * 64 + gq * 16;
        if (base >= F.n) break;                       // uniform across the wavefront
        const int i = base + pi;
        const bool live = i < F.n;
        const int64_t s = F.off + i;
        const float4 p4 = live ? g.p[s] : make_float4(0.f, 0.f, 0.f, 0.f);
        const double px = p4.x, py = p4.y, pz = p4.z;
        // the point's cell, as the per-point stencil computes it
        const int cx = (int)floor((px - (double)F.ox) / c), cy = (int)floor((py - (double)F.oy) / c),
                  cz = (int)floor((pz - (double)F.oz) / c);
        const int x0i = max(cx - 1, 0), x1i = min(cx + 1, F.gx - 1);   // the point's own x-run
        f32x4v acc0 = zero, acc1 = zero, acc2 = zero;
        uint64_t pend = __ballot(live && kk == 0);
        while (pend) {
            const int lead = __builtin_ctzll(pend);
            const int ry = __builtin_amdgcn_readlane(cy, lead), rz = __builtin_amdgcn_readlane(cz, lead);
            const bool inrow = live && ((pend >> pi) & 1) && cy == ry && cz == rz;
            const uint64_t rowm = __ballot(inrow && kk == 0);
            pend &= ~rowm;
            // union of the row's points' x-runs (a point with an empty run adds nothing)
            const bool use = inrow && x0i <= x1i;
            int x0 = use ? x0i : INT_MAX, x1 = use ? x1i : INT_MIN;
            for (int o = 1; o < 16; o <<= 1) {
                x0 = min(x0, __shfl_xor(x0, o, 64));
                x1 = max(x1, __shfl_xor(x1, o, 64));
            }
            x0 = __builtin_amdgcn_readfirstlane(x0);
            x1 = __builtin_amdgcn_readfirstlane(x1);
            if (x0 > x1) continue;
            for (int z = max(rz - 1, 0); z <= min(rz + 1, F.gz - 1); ++z) {
                for (int y = max(ry - 1, 0); y <= min(ry + 1, F.gy - 1); ++y) {
                    const int64_t row = F.cell_off + ((int64_t)z * F.gy + y) * F.gx;
                    const int32_t rb = g.cstart[row + x0], re = g.cstart[row + x1] + g.ccount[row + x1];
                    // Branch-free steps, four per iteration so that their loads are
                    // in flight together: a lane past the run's end reads the run's
                    // last candidate (always in bounds) and adds zero.
                    struct Cand { float4 q; uint32_t w; uint4 t; bool in; };
                    auto fetch = [&](int32_t c0) {
                        const int32_t j = c0 + kk;
                        const int64_t jj = min(j, re - 1);
                        Cand r;
                        r.in = j < re;
                        r.q = g.p[jj];
                        r.w = ((const uint32_t *)(spfh + jj * SPR))[pi];     // bins 2 pi, 2 pi + 1
                        r.t = spfh[jj * SPR + SPR - 1];                       // bin 32 | pad, pad, pad, scale
                        return r;
                    };
                    auto step = [&](const Cand &cd) {
                        const double d2 = pdist2(px, py, pz, (double)cd.q.x, (double)cd.q.y, (double)cd.q.z);
                        const bool hit = cd.in && inrow && d2 > 0.0 && d2 <= r2;
                        // the weight in float32 (v_rsq_f32, within 1 ulp): only the
                        // neighbour decision above needs FP64.  A distance below the
                        // smallest normal float (coincident-looking points) is clamped
                        // there, keeping the weight finite; it dominates the sum either way.
                        const float wv =
                            __builtin_amdgcn_rsqf(fmaxf((float)(hit ? d2 : 1.0), 1.17549435e-38f)) * __uint_as_float(cd.t.w);
                        const float w = hit ? wv : 0.f;
                        // counts need no mask: a lane past the run's end has w = 0, and
                        // slot 33 (taken by pi != 0 for column pi of the third product) is the rows' zero pad
                        const float b0 = (float)(cd.w & 0xffffu), b1 = (float)(cd.w >> 16);
                        const float b2 = (float)(pi == 0 ? (cd.t.x & 0xffffu) : (cd.t.x >> 16));
                        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(w, b0, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(w, b1, acc1, 0, 0, 0);
                        acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(w, b2, acc2, 0, 0, 0);
                    };
                    for (int32_t c0 = rb; c0 < re; c0 += 16) {
                        const Cand A = fetch(c0), B = fetch(c0 + 4), C = fetch(c0 + 8), D = fetch(c0 + 12);
                        step(A);
                        if (c0 + 4 < re) step(B);                 // uniform
                        if (c0 + 8 < re) step(C);
                        if (c0 + 12 < re) step(D);
                    }
                }
            }
        }
        // lane (i, k) holds the sums of points 4 k + r (r < 4), bins 2 i, 2 i + 1 and i + 32
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            red[wv][4 * kk + r][2 * pi] = acc0[r];
            red[wv][4 * kk + r][2 * pi + 1] = acc1[r];
            red[wv][4 * kk + r][pi + 32] = acc2[r];
        }
        wave_sync_lds();
        if (kk == 0 && live) {
            const float *acc = red[wv][pi];
            const int k = knb[s];
            const float ik = k > 0 ? 1.0f / (float)k : 0.0f;
            const uint32_t *si = (const uint32_t *)(spfh + s * SPR);
            const float sci = __uint_as_float(si[4 * SPR - 1]);
            float f[FD];
#pragma unroll
            for (int cc = 0; cc < FD; ++cc)
                f[cc] = (float)((si[cc >> 1] >> (16 * (cc & 1))) & 0xffffu) * sci + acc[cc] * ik;
            bool ok = k >= 1;
#pragma unroll
            for (int blk3 = 0; blk3 < 3; ++blk3) {
                float sum = 0.f;
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) sum += f[NB * blk3 + cc];
                if (sum > 0.f) {
                    const float inv = 1.0f / sum;
#pragma unroll
                    for (int cc = 0; cc < NB; ++cc) f[NB * blk3 + cc] *= inv;
                } else {
                    ok = false;
                }
            }
            const int64_t o = F.off + sorig[s];
            float *dst = Fout + o * FD;
#pragma unroll
            for (int cc = 0; cc < FD; ++cc) dst[cc] = ok ? f[cc] : 0.f;
            valid[o] = ok ? 1 : 0;
            nok += ok ? 1 : 0;
        }
        wave_sync_lds();                              // red is rewritten by the next group
    }
    // per-pair count of valid descriptors
    int t = nok;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) cnt[wv] = t;
    __syncthreads();
    if (threadIdx.x == 0 && ps && F.pair >= 0) {
        const int tot = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        if (tot) atomicAdd(&ps[F.pair].n_valid[b.frag & 1], (unsigned long long)tot);
    }
}

hipError_t launch_fpfh(const GridBufs &g, float r_feature, DescBufs &d, PairState *ps, hipStream_t s) {
    if (g.ntot == 0) return hipSuccess;
    GridView gv{g.cstart, g.ccount, g.sp};
    double r2 = (double)r_feature * (double)r_feature;
    hipLaunchKernelGGL(k_fpfh, dim3(xcd_grid(g.nblk256)), dim3(256), 0, s, (const Frag *)g.frag, (const Blk *)g.blk256,
                       g.nblk256, gv,
                       (const int32_t *)g.sorig, (const uint4 *)d.spfh, (const int32_t *)d.knb, r2, d.F, d.valid, ps);
    return hipGetLastError();
}

}  // namespace lsr
