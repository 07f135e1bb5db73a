// Host runtime behind the C ABI of include/lsr.h.
//
// A call is turned into a plan: the batch's fragment table, block tables,
// consistency-trial table and every scratch array, all in one device
// allocation owned by the plan.  Plans are cached by the call's signature
// (kind, sizes, input/output addresses, parameters), so repeated calls reuse
// their memory and never allocate; a batch plan additionally keeps the HIP
// graph of its launch sequence and replays it.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lsr_internal.h"
#include "match_common.h"

namespace lsr {
int trials_per_block();
int64_t align_blocks(const int64_t *coff, int nprob, void *host_tab, int64_t *pblk);
size_t align_block_bytes();
size_t align_seg_bytes(int64_t m, int64_t nP, int64_t nQ);
hipError_t launch_align(bool bwd, const float *const P[3], int64_t nP, const float *const Q[3], int64_t nQ,
                        const int32_t *corr, int64_t m,
                        const void *dev_tab, int64_t nblocks, const int64_t *dev_pblk, int nprob, const double *T,
                        const double *mu, const double *dE, double *partial, double *out, float *const dP[3],
                        float *const dQ[3], char *seg, hipStream_t s);
hipError_t launch_retract(int n, const double *xi, const double *T, double *Tout, hipStream_t s);
hipError_t launch_retract_grad(int n, const double *xi, const double *gl, double *gx, hipStream_t s);
hipError_t launch_match_bf16(const GridBufs &g, DescBufs &d, MatchBufs &m, PairState *ps, void *scratch, int shape,
                             hipStream_t s);
int screen_shapes();
int consistency_shapes();
size_t voxel_sort_bytes(int64_t n);
size_t voxel_ws_bytes(int64_t n);
hipError_t launch_voxel(const float *const *src_dev, const float *const src[6], int64_t n, float v,
                        float *const *out_dev, int64_t *count, char *ws, size_t sort_bytes, hipStream_t s);
size_t match_bf16_scratch(const GridBufs &g, int64_t pk_rows);
}  // namespace lsr

using namespace lsr;

namespace {

enum PlanKind { K_PAIRS = 1, K_NORMALS, K_FPFH, K_MATCH, K_CONS, K_VERIFY, K_ALIGN, K_VOXEL, K_RANSAC, K_RANSAC_STAGE,
                K_SURFEL, K_EDGE, K_LOOP };

struct FragIn {
    const float *src[6];
    int64_t n;
    int64_t uoff;                  // first point in the caller's cloud
};

struct Plan {
    std::vector<char> key;
    char *dmem = nullptr;
    size_t dbytes = 0;
    char *hmem = nullptr;          // pinned host copy of the tables
    size_t hbytes = 0;
    GridBufs g{};
    DescBufs d{};
    MatchBufs m{};
    PairState *ps = nullptr;
    int npairs = 0;
    TrialBlk *tb = nullptr;
    int ntb = 0;
    int32_t *scan_tmp = nullptr;
    double *nrm_orig = nullptr;    // stage calls: normals in original order (3 per point)
    int64_t *cnt64 = nullptr;      // small device scalars for stage outputs
    void *mscratch = nullptr;      // matcher scratch
    void *extra = nullptr;         // stage-specific scratch (RANSAC hypotheses)
    bool busy = false;             // in use by the current call: never released to make room
    int64_t pk_rows = 0;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    // align-loss tables
    void *atab = nullptr;
    int64_t *apblk = nullptr;
    double *apart = nullptr;
    int64_t anblk = 0;
    ~Plan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (dmem) (void)hipFree(dmem);
        if (hmem) (void)hipHostFree(hmem);
    }
};

struct Layout {                    // sizes of one plan's buffers, in allocation order
    std::vector<size_t> sz;
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = (total + 255) & ~size_t(255);
        sz.push_back(off);
        total = off + bytes;
        return off;
    }
};

}  // namespace

namespace lsr {
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev;
    std::vector<std::string> names;
    size_t used = 0;
};
static Timing g_timing;
void tmark(const char *name, hipStream_t s) {
    Timing &T = g_timing;
    if (!T.on) return;
    if (T.used == T.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        T.ev.push_back(e);
        T.names.push_back("");
    }
    T.names[T.used] = name;
    (void)hipEventRecord(T.ev[T.used], s);
    ++T.used;
}
}  // namespace lsr

struct lsr_ctx {
    int device = 0;
    void *scratch = nullptr;       // this device's address of the allocation-free solve's state (or NULL)
    hipError_t scratch_err = hipSuccess;
    size_t cap = 0;                // workspace cap in bytes (0: none)
    int tune_screen = 0;           // screen shape variant (autotuned)
    int tune_cons = 0;             // consistency block-width variant (autotuned)
    std::string err = "no error";
    std::string tune_cache;        // JSON file of autotune choices, or empty
    std::vector<std::unique_ptr<Plan>> plans;   // most recently used last
};

namespace {

constexpr size_t MAX_PLANS = 48;

int fail(lsr_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(ctx, LSR_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
void put(std::vector<char> &k, const T &v) {
    const char *p = reinterpret_cast<const char *>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

Plan *find_plan(lsr_ctx *c, const std::vector<char> &key) {
    for (size_t i = 0; i < c->plans.size(); ++i)
        if (c->plans[i]->key == key) {
            std::unique_ptr<Plan> p = std::move(c->plans[i]);
            c->plans.erase(c->plans.begin() + i);
            c->plans.push_back(std::move(p));
            return c->plans.back().get();
        }
    return nullptr;
}

bool capturing(hipStream_t s) {
    if (!s) return false;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

int add_plan(lsr_ctx *c, std::unique_ptr<Plan> p, Plan **out) {
    if (c->plans.size() >= MAX_PLANS) {
        HIPCHK(c, hipDeviceSynchronize());
        for (size_t k = 0; k < c->plans.size(); ++k)
            if (!c->plans[k]->busy) { c->plans.erase(c->plans.begin() + (ptrdiff_t)k); break; }
    }
    c->plans.push_back(std::move(p));
    *out = c->plans.back().get();
    return LSR_OK;
}

// Device memory of a new plan under the context's workspace cap: cached plans
// are dropped, least recently used first, until the new block fits; a block
// larger than the cap on its own is LSR_ENOMEM.
int plan_malloc(lsr_ctx *c, Plan *P, size_t bytes) {
    if (c->cap) {
        if (bytes > c->cap)
            return fail(c, LSR_ENOMEM, "workspace of %zu bytes exceeds the context's cap of %zu bytes", bytes, c->cap);
        size_t used = 0;
        for (auto &q : c->plans) used += q->dbytes;
        if (used + bytes > c->cap) {
            HIPCHK(c, hipDeviceSynchronize());
            for (size_t k = 0; k < c->plans.size() && used + bytes > c->cap;) {
                if (c->plans[k]->busy) { ++k; continue; }
                used -= c->plans[k]->dbytes;
                c->plans.erase(c->plans.begin() + (ptrdiff_t)k);
            }
            if (used + bytes > c->cap)
                return fail(c, LSR_ENOMEM, "workspace of %zu bytes does not fit beside the %zu bytes in use (cap %zu)",
                            bytes, used, c->cap);
        }
    }
    hipError_t e = hipMalloc((void **)&P->dmem, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        P->dmem = nullptr;
        return fail(c, e == hipErrorOutOfMemory ? LSR_ENOMEM : LSR_EHIP, "hipMalloc(%zu): %s", bytes,
                    hipGetErrorString(e));
    }
    P->dbytes = bytes;
    return LSR_OK;
}

// cells of a fragment's grid; at least n: the grid build keeps each point's arrival rank in its
// cell in the ncells-long cursor array
int64_t cells_for(int64_t n) { return 4 * n + 4096; }

// Lay out and allocate a fragment-batch plan.  frags[f] are the inputs;
// pairs pair fragment 2b with 2b+1 when `paired`.
int make_batch_plan(lsr_ctx *c, const std::vector<FragIn> &frags, bool paired, const lsr_params *prm,
                    std::vector<char> key, hipStream_t s, Plan **out, size_t extra_bytes = 0) {
    auto P = std::make_unique<Plan>();
    P->key = std::move(key);
    const int nf = (int)frags.size();
    const int npairs = paired ? nf / 2 : 0;
    std::vector<Frag> hf(nf);
    std::vector<Blk> b256, b512;
    std::vector<TrialBlk> tb;
    std::vector<int64_t> foff(nf + 1, 0);
    int64_t ntot = 0, ncells = 0, pk_rows = 0;
    for (int f = 0; f < nf; ++f) {
        Frag &F = hf[f];
        std::memset(&F, 0, sizeof F);
        for (int a = 0; a < 6; ++a) F.src[a] = frags[f].src[a];
        F.off = ntot;
        F.uoff = frags[f].uoff;
        F.n = (int32_t)frags[f].n;
        F.partner = paired ? (f ^ 1) : (nf == 2 ? (f ^ 1) : -1);
        F.pair = paired ? f / 2 : -1;
        F.cell_off = ncells;
        F.cell_cap = (int32_t)cells_for(F.n);
        F.pk_off = pk_rows;
        F.blk256_first = (int32_t)b256.size();
        ntot += F.n;
        ncells += F.cell_cap;
        foff[f + 1] = ntot;
        for (int32_t st = 0; st < F.n; st += 256) b256.push_back(Blk{f, st});
        for (int32_t st = 0; st < F.n; st += 512) b512.push_back(Blk{f, st});
        pk_rows += ((int64_t)F.n + 127) / 128 * 128;
    }
    if (paired && prm) {
        const int tpb = trials_per_block();
        for (int b = 0; b < npairs; ++b) {
            int64_t nP = hf[2 * b].n;
            int64_t T = prm->n_trials > 0 ? prm->n_trials : std::min<int64_t>(4000000, 100 * nP);
            if (nP == 0) T = 0;
            for (int64_t f0 = 0; f0 < T; f0 += tpb) tb.push_back(TrialBlk{b, 0, f0, T});
        }
    }
    int precision = prm ? prm->precision : LSR_FP32;
    P->npairs = npairs;
    P->pk_rows = pk_rows;
    P->g.nfrag = nf;
    P->g.ntot = ntot;
    P->g.ncells = ncells;
    P->g.nblk256 = (int)b256.size();
    P->g.nblk512 = (int)b512.size();
    P->g.pk_rows = pk_rows;
    P->g.max_np = 0;
    for (int f = 0; f < nf; f += 2) P->g.max_np = std::max(P->g.max_np, hf[f].n);
    P->ntb = (int)tb.size();

    // host tables (pinned), copied once
    Layout H;
    size_t h_frag = H.add(sizeof(Frag) * nf), h_b256 = H.add(sizeof(Blk) * b256.size()),
           h_b512 = H.add(sizeof(Blk) * b512.size()), h_tb = H.add(sizeof(TrialBlk) * tb.size()),
           h_foff = H.add(sizeof(int64_t) * (nf + 1));
    // device layout
    Layout D;
    size_t o_tabs = D.add(H.total);
    size_t n1 = (size_t)std::max<int64_t>(ntot, 1), c1 = (size_t)std::max<int64_t>(ncells, 1);
    size_t o_cellpt = D.add(4 * n1), o_cstart = D.add(4 * (c1 + 1)), o_ccount = D.add(4 * c1),
           o_cursor = D.add(4 * (c1 + scan_tmp_elems(ncells))), o_tmp = D.add(4 * n1);
    size_t o_sp = D.add(16 * n1);
    size_t o_s[6];
    for (int a = 3; a < 6; ++a) o_s[a] = D.add(4 * n1);
    size_t o_sorig = D.add(4 * n1);
    size_t o_n[3];
    for (int a = 0; a < 3; ++a) o_n[a] = D.add(8 * n1);
    size_t o_spfh = D.add(16 * SPR * n1), o_knb = D.add(4 * n1), o_F = D.add(4 * FD * n1), o_valid = D.add(4 * n1);
    size_t o_pk = D.add(2 * PK * (size_t)std::max<int64_t>(pk_rows, 1));
    size_t o_cpack = D.add(32 * n1), o_cwords = D.add(sizeof(uint2) * corr_words(ntot, nf));
    size_t o_nnkey = D.add(8 * n1);
    size_t o_nn = D.add(4 * n1), o_dist = D.add(4 * n1), o_mut = D.add(n1), o_flag = D.add(4 * n1),
           o_kpos = D.add(4 * n1), o_kp = D.add(12 * n1), o_kq = D.add(12 * n1), o_ki = D.add(4 * n1);
    size_t o_ps = D.add(sizeof(PairState) * (size_t)std::max(npairs, 1));
    size_t o_stmp = D.add(4 * scan_tmp_elems(ntot));
    size_t o_nrm = D.add(24 * n1);
    size_t o_cnt = D.add(8 * 16);
    size_t msz = precision == LSR_BF16_SCREEN ? match_bf16_scratch(P->g, pk_rows) : 0;
    size_t o_msc = D.add(std::max<size_t>(msz, 256));
    size_t o_extra = D.add(std::max<size_t>(extra_bytes, 256));

    if (capturing(s)) return fail(c, LSR_ENOMEM, "a new plan would allocate while the stream is being captured");
    HIPCHK(c, hipHostMalloc((void **)&P->hmem, std::max<size_t>(H.total, 256), hipHostMallocDefault));
    P->hbytes = H.total;
    int rc0 = plan_malloc(c, P.get(), D.total);
    if (rc0) return rc0;
    char *hb = P->hmem, *db = P->dmem;
    std::memcpy(hb + h_frag, hf.data(), sizeof(Frag) * nf);
    if (!b256.empty()) std::memcpy(hb + h_b256, b256.data(), sizeof(Blk) * b256.size());
    if (!b512.empty()) std::memcpy(hb + h_b512, b512.data(), sizeof(Blk) * b512.size());
    if (!tb.empty()) std::memcpy(hb + h_tb, tb.data(), sizeof(TrialBlk) * tb.size());
    std::memcpy(hb + h_foff, foff.data(), sizeof(int64_t) * (nf + 1));
    char *tabs = db + o_tabs;
    P->g.frag = (Frag *)(tabs + h_frag);
    P->g.blk256 = (Blk *)(tabs + h_b256);
    P->g.blk512 = (Blk *)(tabs + h_b512);
    P->tb = (TrialBlk *)(tabs + h_tb);
    P->g.frag_off = (int64_t *)(tabs + h_foff);
    P->g.cell_of_pt = (int32_t *)(db + o_cellpt);
    P->g.cstart = (int32_t *)(db + o_cstart);
    P->g.ccount = (int32_t *)(db + o_ccount);
    P->g.cursor = (int32_t *)(db + o_cursor);
    P->g.tmp = (int32_t *)(db + o_tmp);
    P->g.sp = (float4 *)(db + o_sp);
    P->g.snx = (float *)(db + o_s[3]); P->g.sny = (float *)(db + o_s[4]); P->g.snz = (float *)(db + o_s[5]);
    P->g.sorig = (int32_t *)(db + o_sorig);
    P->d.nx = (double *)(db + o_n[0]); P->d.ny = (double *)(db + o_n[1]); P->d.nz = (double *)(db + o_n[2]);
    P->d.spfh = (uint4 *)(db + o_spfh);
    P->d.knb = (int32_t *)(db + o_knb);
    P->d.F = (float *)(db + o_F);
    P->d.valid = (int32_t *)(db + o_valid);
    P->d.pk = (uint16_t *)(db + o_pk);
    P->m.nn = (int32_t *)(db + o_nn);
    P->m.nnkey = (unsigned long long *)(db + o_nnkey);
    P->m.dist = (float *)(db + o_dist);
    P->m.mutual = (uint8_t *)(db + o_mut);
    P->m.cpack = (float4 *)(db + o_cpack);
    P->m.cwords = (uint2 *)(db + o_cwords);
    P->m.flag = (int32_t *)(db + o_flag);
    P->m.kpos = (int32_t *)(db + o_kpos);
    P->m.kp = (float *)(db + o_kp);
    P->m.kq = (float *)(db + o_kq);
    P->m.ki = (int32_t *)(db + o_ki);
    P->ps = (PairState *)(db + o_ps);
    P->scan_tmp = (int32_t *)(db + o_stmp);
    P->nrm_orig = (double *)(db + o_nrm);
    P->cnt64 = (int64_t *)(db + o_cnt);
    P->mscratch = db + o_msc;
    P->extra = db + o_extra;
    HIPCHK(c, hipMemcpyAsync(tabs, hb, H.total, hipMemcpyHostToDevice, s));
    return add_plan(c, std::move(P), out);
}

int check_params(lsr_ctx *c, const lsr_params *p) {
    if (!p) return fail(c, LSR_EINVAL, "params is NULL");
    auto fin = [](double v) { return v == v && v < 1e300 && v > -1e300; };
    if (!fin(p->r_normal) || !fin(p->r_feature) || !fin(p->max_corr) || !fin(p->tau) || !fin(p->gnc_div) ||
        !fin(p->min_inlier_ratio) || !fin(p->normal_cos))
        return fail(c, LSR_EINVAL, "non-finite parameter");
    if (!(p->r_normal > 0) || !(p->r_feature > 0) || !(p->max_corr > 0))
        return fail(c, LSR_EINVAL, "radii and max_corr must be positive");
    if (!(p->tau > 0 && p->tau <= 1)) return fail(c, LSR_EINVAL, "tau must lie in (0, 1]");
    if (!(p->gnc_div > 1) || p->gnc_every < 1 || p->gnc_max_iter < 0 || p->polish_iter < 0)
        return fail(c, LSR_EINVAL, "invalid non-convexity schedule");
    if (p->precision != LSR_FP32 && p->precision != LSR_BF16_SCREEN)
        return fail(c, LSR_EINVAL, "unknown precision %d", p->precision);
    if (p->n_trials > (int64_t)1 << 40) return fail(c, LSR_EINVAL, "n_trials too large");
    return LSR_OK;
}

int check_cloud(lsr_ctx *c, const lsr_cloud *cl, const char *name, bool need_normals) {
    if (!cl) return fail(c, LSR_EINVAL, "%s is NULL", name);
    if (cl->n < 0 || cl->n > ((int64_t)1 << 28)) return fail(c, LSR_EINVAL, "%s: size %lld out of range", name, (long long)cl->n);
    if (cl->n > 0 && (!cl->x || !cl->y || !cl->z)) return fail(c, LSR_EINVAL, "%s: NULL coordinates", name);
    if (need_normals && cl->n > 0 && (!cl->nx || !cl->ny || !cl->nz)) return fail(c, LSR_EINVAL, "%s: NULL normals", name);
    return LSR_OK;
}

FragIn frag_of(const lsr_cloud *c, int64_t off, int64_t n) {
    FragIn f;
    const float *a[6] = {c->x, c->y, c->z, c->nx, c->ny, c->nz};
    for (int k = 0; k < 6; ++k) f.src[k] = a[k] ? a[k] + off : nullptr;
    f.n = n;
    f.uoff = off;
    return f;
}

// The full registration sequence over a paired plan.
int run_pairs(lsr_ctx *c, Plan *P, const lsr_params &prm, lsr_result *d_out, hipStream_t s) {
    float r_cell = std::max(std::max(prm.r_normal, prm.r_feature), prm.max_corr);
    tmark("start", s);
    HIPCHK(c, fill<uint32_t>((uint32_t *)P->ps, 0u, (int64_t)(sizeof(PairState) * P->npairs / 4), s));
    HIPCHK(c, build_grids(P->g, r_cell, s));
    tmark("grid", s);
    HIPCHK(c, launch_normals(P->g, prm.r_normal, P->d, nullptr, s));
    tmark("normals", s);
    HIPCHK(c, launch_spfh(P->g, prm.r_feature, P->d, s));
    tmark("spfh", s);
    HIPCHK(c, launch_fpfh(P->g, prm.r_feature, P->d, P->ps, s));
    tmark("fpfh", s);
    if (prm.precision == LSR_BF16_SCREEN) {
        HIPCHK(c, launch_match_bf16(P->g, P->d, P->m, P->ps, P->mscratch, c->tune_screen, s));
        tmark("fallback", s);
    } else {
        HIPCHK(c, launch_match_fp32(P->g, P->d, P->m, s));
        tmark("match_fp32", s);
    }
    HIPCHK(c, launch_mutual(P->g, P->m, P->ps, s));
    HIPCHK(c, launch_consistency(P->g, P->m, P->ps, P->tb, P->ntb, prm.tau, prm.seed, c->tune_cons, P->scan_tmp, s));
    tmark("consistency", s);
    HIPCHK(c, launch_compact(P->g, P->m, P->ps, P->scan_tmp, s));
    HIPCHK(c, launch_gnc(P->g, P->m, P->ps, P->npairs, prm, s));
    tmark("gnc", s);
    HIPCHK(c, launch_verify(P->g, P->d, P->ps, prm.max_corr, prm.normal_check, prm.normal_cos, s));
    HIPCHK(c, launch_finalize(P->g, P->ps, P->npairs, prm, d_out, s));
    tmark("verify", s);
    return LSR_OK;
}

__global__ void k_gnc_info(const PairState *ps, double *T, double *info) {
    if (threadIdx.x < 16) T[threadIdx.x] = ps->T[threadIdx.x];
    if (threadIdx.x == 0) {
        info[0] = ps->status; info[1] = ps->iters; info[2] = ps->mu_final; info[3] = ps->energy;
    }
}

__global__ void k_verify_info(const PairState *ps, const Frag *frag, double delta2, double *info) {
    double n = (double)ps->n_inliers;
    info[0] = n;
    info[1] = frag[0].n > 0 ? n / (double)frag[0].n : 0.0;
    info[2] = ps->n_inliers ? sqrt((double)ps->sum_d2_fixed / 1099511627776.0 * delta2 / n) : 0.0;
}

__global__ void k_set_T(PairState *ps, const double *T) {
    if (threadIdx.x < 16) ps->T[threadIdx.x] = T[threadIdx.x];
}

__global__ void k_flag_out(const int32_t *flag, int64_t n, uint8_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = flag[i] ? 1 : 0;
}

__global__ void k_passed_out(const PairState *ps, int64_t *out) { *out = (int64_t)ps->trials_passed; }

__global__ void k_fallback_out(const PairState *ps, int64_t *out) { *out = (int64_t)ps->n_fallback; }

// Per-point intermediate results of a paired plan, scattered to the caller's
// point order: every point gets its descriptor (33 floats, zero when invalid)
// and validity; P points get their descriptor neighbour in Q, the reciprocal
// flag and the consistency flag; Q points their neighbour in P.
__global__ void __launch_bounds__(256) k_trace_out(const Frag *frag, const Blk *blk, const int32_t *nn,
                                                   const uint8_t *mutual, const int32_t *flag, const float *F,
                                                   const int32_t *valid, lsr_trace tr) {
    const Blk b = blk[blockIdx.x];
    const Frag &Fr = frag[b.frag];
    const int i = b.start + threadIdx.x;
    if (i >= Fr.n || Fr.partner < 0) return;
    const int64_t g = Fr.off + i, u = Fr.uoff + i;
    const bool q = b.frag & 1;
    float *desc = q ? tr.desc_Q : tr.desc_P;
    int32_t *val = q ? tr.valid_Q : tr.valid_P;
    if (desc)
        for (int c = 0; c < FD; ++c) desc[u * FD + c] = F[g * FD + c];
    if (val) val[u] = valid[g];
    if (q) {
        if (tr.nnP) tr.nnP[u] = nn[g];
    } else {
        if (tr.nnQ) tr.nnQ[u] = nn[g];
        if (tr.mutual) tr.mutual[u] = mutual[g];
        if (tr.consistent) tr.consistent[u] = flag[g] ? 1 : 0;
    }
}

unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================

extern "C" {

int lsr_set_timing(lsr_ctx *ctx, int enable) {
    if (!ctx) return LSR_EINVAL;
    g_timing.on = enable != 0;
    g_timing.used = 0;
    return LSR_OK;
}

int lsr_get_timing(lsr_ctx *ctx, int max_steps, char *names, double *ms, int *n_steps) {
    if (!ctx || !n_steps || max_steps < 0) return LSR_EINVAL;
    Timing &T = g_timing;
    HIPCHK(ctx, hipDeviceSynchronize());
    int n = (int)T.used > 0 ? (int)T.used - 1 : 0;
    if (n > max_steps) n = max_steps;
    for (int k = 0; k < n; ++k) {
        float t = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t, T.ev[k], T.ev[k + 1]));
        if (ms) ms[k] = t;
        if (names) { std::strncpy(names + 32 * k, T.names[k + 1].c_str(), 31); names[32 * k + 31] = 0; }
    }
    *n_steps = n;
    T.used = 0;
    return LSR_OK;
}

void lsr_default_params(lsr_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->r_normal = 0.025f;
    p->r_feature = 0.05f;
    p->max_corr = 0.015f;
    p->tau = 0.9f;
    p->n_trials = 0;
    p->gnc_div = 1.4;
    p->gnc_every = 4;
    p->gnc_max_iter = 256;
    p->polish_iter = 32;
    p->min_inlier_ratio = 0.25f;
    p->min_consistent = 10;
    p->normal_check = 0;
    p->normal_cos = 0.8660254f;
    p->precision = LSR_FP32;
    p->seed = 0x1801015720ULL;
}

}  // extern "C"

// State of the allocation-free pose solve (lsr_stage_gnc_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel: it uses the device
// address hipGetSymbolAddress returns for the current device, looked up once
// per device when the first context on it is created.
constexpr size_t NOALLOC_SCRATCH_BYTES = 1024;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static_assert(sizeof(PairState) <= NOALLOC_SCRATCH_BYTES, "the solve's state must fit the static scratch");

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_addr;     // per device; NULL until looked up

// The calling thread's current device must be `device`.
hipError_t scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) { (void)hipGetLastError(); *out = nullptr; return e; }
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}
}  // namespace

extern "C" {

int lsr_create(lsr_ctx **ctx, int device, size_t workspace_cap_bytes) {
    if (!ctx) return LSR_EINVAL;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LSR_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return LSR_EHIP;
    lsr_ctx *c = new lsr_ctx;
    c->device = device;
    c->cap = workspace_cap_bytes;
    c->scratch_err = scratch_address(device, &c->scratch);
    *ctx = c;
    return LSR_OK;
}

void lsr_destroy(lsr_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->plans.clear();
    delete ctx;
}

const char *lsr_last_error(const lsr_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int lsr_register_pair(lsr_ctx *ctx, const lsr_cloud *P, const lsr_cloud *Q, const lsr_params *prm,
                      lsr_result *d_out, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_params(ctx, prm)) || (rc = check_cloud(ctx, P, "P", true)) || (rc = check_cloud(ctx, Q, "Q", true)))
        return rc;
    if (!d_out) return fail(ctx, LSR_EINVAL, "d_out is NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<FragIn> fr = {frag_of(P, 0, P->n), frag_of(Q, 0, Q->n)};
    std::vector<char> key;
    put(key, (int)K_PAIRS);
    put(key, *prm);
    for (auto &f : fr) { put(key, f.n); for (int a = 0; a < 6; ++a) put(key, f.src[a]); }
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, prm, key, s, &pl))) return rc;
    return run_pairs(ctx, pl, *prm, d_out, s);
}

}  // extern "C"

namespace {
// Checks a batch call's arguments and lists its fragments (P_b, Q_b per pair).
int batch_frags(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all, const int64_t *offP, const int64_t *offQ,
                int32_t n_pairs, const lsr_params *prm, std::vector<FragIn> &fr) {
    int rc;
    if ((rc = check_params(ctx, prm)) || (rc = check_cloud(ctx, P_all, "P_all", true)) ||
        (rc = check_cloud(ctx, Q_all, "Q_all", true)))
        return rc;
    if (n_pairs < 0 || n_pairs > (1 << 20)) return fail(ctx, LSR_EINVAL, "n_pairs %d out of range", n_pairs);
    if (n_pairs == 0) return LSR_OK;
    if (!offP || !offQ) return fail(ctx, LSR_EINVAL, "NULL offsets");
    for (int b = 0; b < n_pairs; ++b) {
        if (offP[b] < 0 || offP[b + 1] < offP[b] || offP[b + 1] > P_all->n || offQ[b] < 0 || offQ[b + 1] < offQ[b] ||
            offQ[b + 1] > Q_all->n)
            return fail(ctx, LSR_EINVAL, "bad offsets at pair %d", b);
    }
    fr.clear();
    fr.reserve(2 * n_pairs);
    for (int b = 0; b < n_pairs; ++b) {
        fr.push_back(frag_of(P_all, offP[b], offP[b + 1] - offP[b]));
        fr.push_back(frag_of(Q_all, offQ[b], offQ[b + 1] - offQ[b]));
    }
    return LSR_OK;
}

// Drops every cached plan (their graphs hold the previous kernel variants).
int drop_plans(lsr_ctx *c) {
    HIPCHK(c, hipDeviceSynchronize());
    c->plans.clear();
    return LSR_OK;
}

// Mean time of `reps` runs of fn on stream s (one untimed run first).
template <class Fn>
int time_ms(lsr_ctx *c, hipStream_t s, int reps, Fn &&fn, float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(c, LSR_EHIP, "hipEventCreate"); }
    int rc = fn();
    hipError_t e = hipSuccess;
    if (!rc) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && !rc && e == hipSuccess; ++r) rc = fn();
    if (!rc && e == hipSuccess) e = hipEventRecord(e1, s);
    if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (!rc && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess) return fail(c, LSR_EHIP, "timing: %s", hipGetErrorString(e));
    *ms = t / (float)reps;
    return LSR_OK;
}
}  // namespace

extern "C" {

}  // extern "C"

namespace {
// lsr_register_batch; *used receives the plan that ran.
int register_batch_plan(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all, const int64_t *offP,
                        const int64_t *offQ, int32_t n_pairs, const lsr_params *prm, lsr_result *d_out, void *stream,
                        Plan **used) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    std::vector<FragIn> fr;
    if ((rc = batch_frags(ctx, P_all, Q_all, offP, offQ, n_pairs, prm, fr))) return rc;
    if (n_pairs == 0) return LSR_OK;
    if (!d_out) return fail(ctx, LSR_EINVAL, "NULL output");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<char> key;
    put(key, (int)K_PAIRS + 100);
    put(key, *prm);
    put(key, d_out);
    for (auto &f : fr) { put(key, f.n); put(key, f.uoff); for (int a = 0; a < 6; ++a) put(key, f.src[a]); }
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, prm, key, s, &pl))) return rc;
    if (used) *used = pl;
    if (!s || capturing(s) || g_timing.on) return run_pairs(ctx, pl, *prm, d_out, s);   // eager
    if (!pl->gexec) {
        HIPCHK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc = run_pairs(ctx, pl, *prm, d_out, s);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(s, &gr);
        if (rc) { if (gr) (void)hipGraphDestroy(gr); return rc; }
        if (e != hipSuccess) return fail(ctx, LSR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        pl->graph = gr;
        HIPCHK(ctx, hipGraphInstantiate(&pl->gexec, gr, nullptr, nullptr, 0));
    }
    HIPCHK(ctx, hipGraphLaunch(pl->gexec, s));
    return LSR_OK;
}
}  // namespace

extern "C" {

int lsr_register_batch(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all, const int64_t *offP,
                       const int64_t *offQ, int32_t n_pairs, const lsr_params *prm, lsr_result *d_out, void *stream) {
    return register_batch_plan(ctx, P_all, Q_all, offP, offQ, n_pairs, prm, d_out, stream, nullptr);
}

int lsr_register_batch_trace(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all, const int64_t *offP,
                             const int64_t *offQ, int32_t n_pairs, const lsr_params *prm, lsr_result *d_out,
                             const lsr_trace *tr, void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (!tr) return fail(ctx, LSR_EINVAL, "NULL trace");
    Plan *pl = nullptr;
    int rc = register_batch_plan(ctx, P_all, Q_all, offP, offQ, n_pairs, prm, d_out, stream, &pl);
    if (rc || !pl || pl->g.nblk256 == 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_trace_out, dim3(pl->g.nblk256), dim3(256), 0, s, (const Frag *)pl->g.frag,
                       (const Blk *)pl->g.blk256, (const int32_t *)pl->m.nn, (const uint8_t *)pl->m.mutual,
                       (const int32_t *)pl->m.flag, (const float *)pl->d.F, (const int32_t *)pl->d.valid, *tr);
    HIPCHK(ctx, hipGetLastError());
    return LSR_OK;
}

int lsr_get_tune(lsr_ctx *ctx, lsr_tune *out) {
    if (!ctx || !out) return LSR_EINVAL;
    std::memset(out, 0, sizeof *out);
    out->screen_shape = ctx->tune_screen;
    out->consistency_shape = ctx->tune_cons;
    out->n_screen_shapes = screen_shapes();
    out->n_consistency_shapes = consistency_shapes();
    return LSR_OK;
}

int lsr_set_tune(lsr_ctx *ctx, const lsr_tune *t) {
    if (!ctx || !t) return LSR_EINVAL;
    if (t->screen_shape < 0 || t->screen_shape >= screen_shapes() || t->consistency_shape < 0 ||
        t->consistency_shape >= consistency_shapes())
        return fail(ctx, LSR_EINVAL, "tune variant out of range");
    if (t->screen_shape == ctx->tune_screen && t->consistency_shape == ctx->tune_cons) return LSR_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    int rc;
    if ((rc = drop_plans(ctx))) return rc;
    ctx->tune_screen = t->screen_shape;
    ctx->tune_cons = t->consistency_shape;
    return LSR_OK;
}

}  // extern "C"

// ---- the tune cache: one JSON object per line inside an "entries" array
namespace {

std::string tune_key(lsr_ctx *ctx, const std::vector<FragIn> &fr, int32_t n_pairs) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
    }
    auto p2 = [](int64_t v) { int64_t b = 1; while (b < v) b <<= 1; return b; };
    int64_t tot = 0, mx = 0;
    for (auto &f : fr) { tot += f.n; mx = std::max(mx, f.n); }
    const int64_t mean = fr.empty() ? 0 : (tot + (int64_t)fr.size() - 1) / (int64_t)fr.size();
    char buf[256];
    snprintf(buf, sizeof buf, "%s|pairs=%lld|mean=%lld|max=%lld", arch.c_str(), (long long)p2(n_pairs),
             (long long)p2(mean), (long long)p2(mx));
    return buf;
}

struct TuneEntry {
    std::string key;
    int screen = -1, cons = -1;
    std::string line;
};

std::vector<TuneEntry> read_tune_cache(const std::string &path) {
    std::vector<TuneEntry> out;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return out;
    char buf[4096];
    while (fgets(buf, sizeof buf, f)) {
        std::string l(buf);
        const size_t k = l.find("\"key\": \""), a = l.find("\"screen_shape\": "), b = l.find("\"consistency_shape\": ");
        if (k == std::string::npos || a == std::string::npos || b == std::string::npos) continue;
        const size_t ke = l.find('"', k + 8);
        if (ke == std::string::npos) continue;
        TuneEntry e;
        e.key = l.substr(k + 8, ke - (k + 8));
        e.screen = atoi(l.c_str() + a + 16);
        e.cons = atoi(l.c_str() + b + 21);
        while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == '\r')) l.pop_back();
        e.line = l;
        out.push_back(e);
    }
    fclose(f);
    return out;
}

bool write_tune_cache(const std::string &path, const std::vector<TuneEntry> &es) {
    const std::string tmp = path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\"lsr_tune_cache\": 1, \"entries\": [\n");
    for (size_t k = 0; k < es.size(); ++k) fprintf(f, "%s%s\n", es[k].line.c_str(), k + 1 < es.size() ? "," : "");
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

extern "C" {

int lsr_set_tune_cache(lsr_ctx *ctx, const char *path) {
    if (!ctx) return LSR_EINVAL;
    ctx->tune_cache = path ? path : "";
    return LSR_OK;
}

int lsr_autotune(lsr_ctx *ctx, const lsr_cloud *P_all, const lsr_cloud *Q_all, const int64_t *offP,
                 const int64_t *offQ, int32_t n_pairs, const lsr_params *prm, int32_t reps, lsr_tune *out,
                 void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (reps < 1 || reps > 1000) return fail(ctx, LSR_EINVAL, "reps %d out of range", reps);
    if (screen_shapes() > LSR_MAX_VARIANTS || consistency_shapes() > LSR_MAX_VARIANTS)
        return fail(ctx, LSR_EINVAL, "too many variants");
    int rc;
    std::vector<FragIn> fr;
    if ((rc = batch_frags(ctx, P_all, Q_all, offP, offQ, n_pairs, prm, fr))) return rc;
    if (n_pairs == 0) return fail(ctx, LSR_EINVAL, "autotuning needs at least one pair");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return fail(ctx, LSR_EINVAL, "autotuning cannot run under stream capture");
    lsr_tune res;
    std::memset(&res, 0, sizeof res);
    res.n_screen_shapes = screen_shapes();
    res.n_consistency_shapes = consistency_shapes();
    std::string tkey;
    std::vector<TuneEntry> cache;
    if (!ctx->tune_cache.empty()) {
        tkey = tune_key(ctx, fr, n_pairs);
        cache = read_tune_cache(ctx->tune_cache);
        for (auto &e : cache)
            if (e.key == tkey && e.screen >= 0 && e.screen < res.n_screen_shapes && e.cons >= 0 &&
                e.cons < res.n_consistency_shapes) {
                res.screen_shape = e.screen;
                res.consistency_shape = e.cons;
                res.from_cache = 1;
                if ((rc = lsr_set_tune(ctx, &res))) return rc;
                if (out) *out = res;
                return LSR_OK;
            }
    }
    lsr_params tp = *prm;
    tp.precision = LSR_BF16_SCREEN;                 // the screen is one of the tuned kernels
    const bool timing = g_timing.on;
    g_timing.on = false;
    lsr_result *d_out = nullptr;
    Plan *pl = nullptr;
    std::vector<char> key;
    put(key, (int)K_PAIRS + 200);
    put(key, tp);
    for (auto &f : fr) { put(key, f.n); for (int a = 0; a < 6; ++a) put(key, f.src[a]); }
    pl = find_plan(ctx, key);
    if (!pl) rc = make_batch_plan(ctx, fr, true, &tp, key, s, &pl);
    if (!rc && hipMalloc((void **)&d_out, sizeof(lsr_result) * (size_t)n_pairs) != hipSuccess)
        rc = fail(ctx, LSR_ENOMEM, "autotune output");
    if (!rc) rc = run_pairs(ctx, pl, tp, d_out, s);   // every buffer the tuned stages read
    for (int v = 0; v < res.n_screen_shapes && !rc; ++v)
        rc = time_ms(ctx, s, reps, [&]() -> int {
            HIPCHK(ctx, launch_match_bf16(pl->g, pl->d, pl->m, pl->ps, pl->mscratch, v, s));
            return LSR_OK;
        }, &res.screen_ms[v]);
    for (int v = 0; v < res.n_consistency_shapes && !rc; ++v)
        rc = time_ms(ctx, s, reps, [&]() -> int {
            HIPCHK(ctx, launch_consistency(pl->g, pl->m, pl->ps, pl->tb, pl->ntb, tp.tau, tp.seed, v, pl->scan_tmp, s));
            return LSR_OK;
        }, &res.consistency_ms[v]);
    g_timing.on = timing;
    if (d_out) { (void)hipStreamSynchronize(s); (void)hipFree(d_out); }
    if (rc) return rc;
    for (int v = 1; v < res.n_screen_shapes; ++v)
        if (res.screen_ms[v] < res.screen_ms[res.screen_shape]) res.screen_shape = v;
    for (int v = 1; v < res.n_consistency_shapes; ++v)
        if (res.consistency_ms[v] < res.consistency_ms[res.consistency_shape]) res.consistency_shape = v;
    if ((rc = lsr_set_tune(ctx, &res))) return rc;
    if (!tkey.empty()) {
        TuneEntry e;
        e.key = tkey;
        std::string ms;
        char buf[64];
        for (int v = 0; v < res.n_screen_shapes; ++v) { snprintf(buf, sizeof buf, "%s%.3f", v ? ", " : "", res.screen_ms[v]); ms += buf; }
        std::string mc;
        for (int v = 0; v < res.n_consistency_shapes; ++v) { snprintf(buf, sizeof buf, "%s%.3f", v ? ", " : "", res.consistency_ms[v]); mc += buf; }
        e.line = "{\"key\": \"" + tkey + "\", \"screen_shape\": " + std::to_string(res.screen_shape) +
                 ", \"consistency_shape\": " + std::to_string(res.consistency_shape) + ", \"screen_ms\": [" + ms +
                 "], \"consistency_ms\": [" + mc + "]}";
        std::vector<TuneEntry> keep;
        for (auto &c : cache)
            if (c.key != tkey) keep.push_back(c);
        keep.push_back(e);
        if (!write_tune_cache(ctx->tune_cache, keep))
            return fail(ctx, LSR_EINVAL, "cannot write the tune cache %s", ctx->tune_cache.c_str());
    }
    if (out) *out = res;
    return LSR_OK;
}

int lsr_stage_normals(lsr_ctx *ctx, const lsr_cloud *c, float r_normal, double *d_nrm, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_cloud(ctx, c, "cloud", true))) return rc;
    if (!d_nrm || !(r_normal > 0)) return fail(ctx, LSR_EINVAL, "bad normals arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<FragIn> fr = {frag_of(c, 0, c->n)};
    std::vector<char> key;
    put(key, (int)K_NORMALS);
    put(key, fr[0]);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, false, nullptr, key, s, &pl))) return rc;
    HIPCHK(ctx, build_grids(pl->g, r_normal, s));
    HIPCHK(ctx, launch_normals(pl->g, r_normal, pl->d, d_nrm, s));
    return LSR_OK;
}

int lsr_stage_fpfh(lsr_ctx *ctx, const lsr_cloud *c, const double *d_nrm, float r_feature, float *d_F,
                   int32_t *d_valid, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_cloud(ctx, c, "cloud", false))) return rc;
    if (!d_nrm || !d_F || !d_valid || !(r_feature > 0)) return fail(ctx, LSR_EINVAL, "bad fpfh arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<FragIn> fr = {frag_of(c, 0, c->n)};
    std::vector<char> key;
    put(key, (int)K_FPFH);
    put(key, fr[0]);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, false, nullptr, key, s, &pl))) return rc;
    HIPCHK(ctx, build_grids(pl->g, r_feature, s));
    HIPCHK(ctx, launch_normals_inject(pl->g, d_nrm, pl->d, s));
    HIPCHK(ctx, launch_spfh(pl->g, r_feature, pl->d, s));
    HIPCHK(ctx, launch_fpfh(pl->g, r_feature, pl->d, nullptr, s));
    HIPCHK(ctx, copy<float>(d_F, pl->d.F, c->n * FD, s));
    HIPCHK(ctx, copy<int32_t>(d_valid, pl->d.valid, c->n, s));
    return LSR_OK;
}

int lsr_stage_spfh(lsr_ctx *ctx, const lsr_cloud *c, const double *d_nrm, float r_feature, float *d_spfh,
                   int32_t *d_k, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_cloud(ctx, c, "cloud", false))) return rc;
    if (!d_nrm || !d_spfh || !d_k || !(r_feature > 0)) return fail(ctx, LSR_EINVAL, "bad spfh arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<FragIn> fr = {frag_of(c, 0, c->n)};
    std::vector<char> key;
    put(key, (int)K_FPFH + 1000);
    put(key, fr[0]);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, false, nullptr, key, s, &pl))) return rc;
    HIPCHK(ctx, build_grids(pl->g, r_feature, s));
    HIPCHK(ctx, launch_normals_inject(pl->g, d_nrm, pl->d, s));
    HIPCHK(ctx, launch_spfh(pl->g, r_feature, pl->d, s));
    HIPCHK(ctx, launch_spfh_out(pl->g, pl->d, d_spfh, d_k, s));
    return LSR_OK;
}

int lsr_stage_match(lsr_ctx *ctx, const float *d_F, const int32_t *d_vF, int64_t nP, const float *d_G,
                    const int32_t *d_vG, int64_t nQ, int32_t precision, int32_t *d_nnQ, float *d_dQ,
                    int32_t *d_nnP, float *d_dP, int64_t *d_fallback, void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (nP < 0 || nQ < 0 || nP > (1 << 28) || nQ > (1 << 28)) return fail(ctx, LSR_EINVAL, "bad sizes");
    if ((nP && (!d_F || !d_vF || !d_nnQ || !d_dQ)) || (nQ && (!d_G || !d_vG || !d_nnP || !d_dP)))
        return fail(ctx, LSR_EINVAL, "NULL match argument");
    if (precision != LSR_FP32 && precision != LSR_BF16_SCREEN) return fail(ctx, LSR_EINVAL, "unknown precision");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    FragIn a{}, b{};
    a.n = nP; b.n = nQ;
    std::vector<FragIn> fr = {a, b};
    lsr_params prm;
    lsr_default_params(&prm);
    prm.precision = precision;
    prm.n_trials = 1;
    std::vector<char> key;
    put(key, (int)K_MATCH);
    put(key, nP); put(key, nQ); put(key, precision);
    int rc;
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, &prm, key, s, &pl))) return rc;
    HIPCHK(ctx, fill<uint32_t>((uint32_t *)pl->ps, 0u, (int64_t)(sizeof(PairState) / 4), s));
    HIPCHK(ctx, copy<float>(pl->d.F, d_F, nP * FD, s));
    HIPCHK(ctx, copy<float>(pl->d.F + nP * FD, d_G, nQ * FD, s));
    HIPCHK(ctx, copy<int32_t>(pl->d.valid, d_vF, nP, s));
    HIPCHK(ctx, copy<int32_t>(pl->d.valid + nP, d_vG, nQ, s));
    if (precision == LSR_BF16_SCREEN) {
        HIPCHK(ctx, launch_match_bf16(pl->g, pl->d, pl->m, pl->ps, pl->mscratch, ctx->tune_screen, s));
    } else {
        HIPCHK(ctx, launch_match_fp32(pl->g, pl->d, pl->m, s));
    }
    HIPCHK(ctx, copy<int32_t>(d_nnQ, pl->m.nn, nP, s));
    HIPCHK(ctx, copy<float>(d_dQ, pl->m.dist, nP, s));
    HIPCHK(ctx, copy<int32_t>(d_nnP, pl->m.nn + nP, nQ, s));
    HIPCHK(ctx, copy<float>(d_dP, pl->m.dist + nP, nQ, s));
    if (d_fallback) {
        hipLaunchKernelGGL(k_fallback_out, dim3(1), dim3(1), 0, s, (const PairState *)pl->ps, d_fallback);
        HIPCHK(ctx, hipGetLastError());
    }
    return LSR_OK;
}

int lsr_stage_consistency(lsr_ctx *ctx, const lsr_cloud *P, const lsr_cloud *Q, const int32_t *d_nnQ,
                          const uint8_t *d_mutual, int64_t n_trials, float tau, uint64_t seed, uint8_t *d_flag,
                          int64_t *d_passed, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_cloud(ctx, P, "P", false)) || (rc = check_cloud(ctx, Q, "Q", false))) return rc;
    if (!d_nnQ || !d_mutual || !d_flag || !d_passed || !(tau > 0 && tau <= 1))
        return fail(ctx, LSR_EINVAL, "bad consistency arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<FragIn> fr = {frag_of(P, 0, P->n), frag_of(Q, 0, Q->n)};
    lsr_params prm;
    lsr_default_params(&prm);
    prm.n_trials = n_trials;
    prm.tau = tau;
    std::vector<char> key;
    put(key, (int)K_CONS);
    put(key, n_trials);
    for (auto &f : fr) put(key, f);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, &prm, key, s, &pl))) return rc;
    HIPCHK(ctx, fill<uint32_t>((uint32_t *)pl->ps, 0u, (int64_t)(sizeof(PairState) / 4), s));
    HIPCHK(ctx, copy<int32_t>(pl->m.nn, d_nnQ, P->n, s));
    HIPCHK(ctx, copy<uint8_t>(pl->m.mutual, d_mutual, P->n, s));
    HIPCHK(ctx, launch_consistency(pl->g, pl->m, pl->ps, pl->tb, pl->ntb, tau, seed, ctx->tune_cons, pl->scan_tmp, s));
    if (P->n > 0) {
        hipLaunchKernelGGL(k_flag_out, dim3(nblk(P->n, 256)), dim3(256), 0, s, (const int32_t *)pl->m.flag, P->n, d_flag);
        HIPCHK(ctx, hipGetLastError());
    }
    hipLaunchKernelGGL(k_passed_out, dim3(1), dim3(1), 0, s, (const PairState *)pl->ps, d_passed);
    HIPCHK(ctx, hipGetLastError());
    return LSR_OK;
}

int lsr_stage_gnc(lsr_ctx *ctx, const double *d_p, const double *d_q, int64_t m, const lsr_params *prm, double *d_T,
                  double *d_info, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_params(ctx, prm))) return rc;
    if (m < 0 || (m > 0 && (!d_p || !d_q)) || !d_T || !d_info) return fail(ctx, LSR_EINVAL, "bad gnc arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<char> key;
    put(key, (int)K_ALIGN + 50);
    Plan *pl = find_plan(ctx, key);
    if (!pl) {
        auto P = std::make_unique<Plan>();
        P->key = key;
        if (capturing(s)) return fail(ctx, LSR_ENOMEM, "allocation during capture");
        if ((rc = plan_malloc(ctx, P.get(), sizeof(PairState)))) return rc;
        P->ps = (PairState *)P->dmem;
        if ((rc = add_plan(ctx, std::move(P), &pl))) return rc;
    }
    HIPCHK(ctx, launch_gnc_direct(d_p, d_q, m, *prm, pl->ps, s));
    hipLaunchKernelGGL(k_gnc_info, dim3(1), dim3(64), 0, s, (const PairState *)pl->ps, d_T, d_info);
    HIPCHK(ctx, hipGetLastError());
    return LSR_OK;
}

int lsr_stage_gnc_noalloc(lsr_ctx *ctx, const double *d_p, const double *d_q, int64_t m, const lsr_params *prm,
                          double *d_T, double *d_info, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_params(ctx, prm))) return rc;
    if (m < 0 || (m > 0 && (!d_p || !d_q)) || !d_T || !d_info) return fail(ctx, LSR_EINVAL, "bad gnc arguments");
    if (!ctx->scratch)
        return fail(ctx, LSR_EHIP, "static scratch of device %d unavailable: hipGetSymbolAddress: %s", ctx->device,
                    hipGetErrorString(ctx->scratch_err));
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    PairState *st = (PairState *)ctx->scratch;      // every output field is written by the solve
    HIPCHK(ctx, launch_gnc_direct(d_p, d_q, m, *prm, st, s));
    hipLaunchKernelGGL(k_gnc_info, dim3(1), dim3(64), 0, s, (const PairState *)st, d_T, d_info);
    HIPCHK(ctx, hipGetLastError());
    return LSR_OK;
}

int lsr_stage_verify(lsr_ctx *ctx, const lsr_cloud *P, const double *d_nrmP, const lsr_cloud *Q,
                     const double *d_nrmQ, const double *d_T, float delta, int32_t normal_check, float normal_cos,
                     double *d_info, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_cloud(ctx, P, "P", false)) || (rc = check_cloud(ctx, Q, "Q", false))) return rc;
    if (!d_T || !d_info || !(delta > 0) || (normal_check && (!d_nrmP || !d_nrmQ)))
        return fail(ctx, LSR_EINVAL, "bad verify arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<FragIn> fr = {frag_of(P, 0, P->n), frag_of(Q, 0, Q->n)};
    std::vector<char> key;
    put(key, (int)K_VERIFY);
    for (auto &f : fr) put(key, f);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, nullptr, key, s, &pl))) return rc;
    HIPCHK(ctx, fill<uint32_t>((uint32_t *)pl->ps, 0u, (int64_t)(sizeof(PairState) / 4), s));
    HIPCHK(ctx, build_grids(pl->g, delta, s));
    if (normal_check) {
        HIPCHK(ctx, copy<double>(pl->nrm_orig, d_nrmP, 3 * P->n, s));
        HIPCHK(ctx, copy<double>(pl->nrm_orig + 3 * P->n, d_nrmQ, 3 * Q->n, s));
        HIPCHK(ctx, launch_normals_inject(pl->g, pl->nrm_orig, pl->d, s));
    }
    hipLaunchKernelGGL(k_set_T, dim3(1), dim3(64), 0, s, pl->ps, d_T);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, launch_verify(pl->g, pl->d, pl->ps, delta, normal_check, normal_cos, s));
    hipLaunchKernelGGL(k_verify_info, dim3(1), dim3(1), 0, s, (const PairState *)pl->ps, (const Frag *)pl->g.frag,
                       (double)delta * (double)delta, d_info);
    HIPCHK(ctx, hipGetLastError());
    return LSR_OK;
}

int lsr_voxel_downsample(lsr_ctx *ctx, const lsr_cloud *c, float voxel, float *const out[6], int64_t *d_count,
                         void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_cloud(ctx, c, "cloud", true))) return rc;
    if (!(voxel > 0) || !(voxel < 1e30f) || !out || !d_count) return fail(ctx, LSR_EINVAL, "bad voxel arguments");
    for (int a = 0; a < 6; ++a)
        if (!out[a] && c->n > 0) return fail(ctx, LSR_EINVAL, "NULL output array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (c->n == 0) {
        HIPCHK(ctx, fill<int64_t>(d_count, 0, 1, s));
        return LSR_OK;
    }
    std::vector<char> key;
    put(key, (int)K_VOXEL);
    put(key, c->n);
    const float *src[6] = {c->x, c->y, c->z, c->nx, c->ny, c->nz};
    for (int a = 0; a < 6; ++a) put(key, src[a]);
    for (int a = 0; a < 6; ++a) put(key, out[a]);
    Plan *pl = find_plan(ctx, key);
    if (!pl) {
        auto P = std::make_unique<Plan>();
        P->key = key;
        size_t ws = voxel_ws_bytes(c->n);
        if (capturing(s)) return fail(ctx, LSR_ENOMEM, "allocation during capture");
        if ((rc = plan_malloc(ctx, P.get(), ws + 256))) return rc;
        HIPCHK(ctx, hipHostMalloc((void **)&P->hmem, 256, hipHostMallocDefault));
        std::memcpy(P->hmem, src, sizeof(src));
        std::memcpy(P->hmem + 64, out, 6 * sizeof(float *));
        HIPCHK(ctx, hipMemcpyAsync(P->dmem + ws, P->hmem, 128, hipMemcpyHostToDevice, s));
        if ((rc = add_plan(ctx, std::move(P), &pl))) return rc;
    }
    const size_t ws = voxel_ws_bytes(c->n);
    const float *const *src_dev = (const float *const *)(pl->dmem + ws);
    float *const *out_dev = (float *const *)(pl->dmem + ws + 64);
    HIPCHK(ctx, launch_voxel(src_dev, src, c->n, voxel, out_dev, d_count, pl->dmem, voxel_sort_bytes(c->n), s));
    return LSR_OK;
}

int lsr_surfel_correct(lsr_ctx *ctx, const float *const surfels[6], const int32_t *d_t0, const int32_t *d_tu,
                       int64_t n, const double *h_T_old, const double *h_T_new, const int32_t *h_t_kf,
                       int32_t n_kf, const lsr_camera *cam, float *const out[6], int32_t *d_new_index,
                       int32_t *d_k_obs, int64_t *d_n_kept, void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (n < 0 || n > INT32_MAX) return fail(ctx, LSR_EINVAL, "surfel count %lld out of range", (long long)n);
    if (n_kf < 0 || n_kf > (1 << 20)) return fail(ctx, LSR_EINVAL, "keyframe count %d out of range", n_kf);
    if (!cam || !d_n_kept || (n > 0 && (!surfels || !d_t0 || !d_tu || !out)) ||
        (n_kf > 0 && (!h_T_old || !h_T_new || !h_t_kf)))
        return fail(ctx, LSR_EINVAL, "NULL surfel-correction argument");
    for (int a = 0; a < 6 && n > 0; ++a)
        if (!surfels[a] || !out[a]) return fail(ctx, LSR_EINVAL, "NULL surfel array");
    const double cp[6] = {cam->fx, cam->fy, cam->cx, cam->cy, cam->z_min, cam->z_max};
    for (double v : cp)
        if (!std::isfinite(v)) return fail(ctx, LSR_EINVAL, "non-finite camera parameter");
    if (cam->width <= 0 || cam->height <= 0) return fail(ctx, LSR_EINVAL, "bad image size");
    for (int32_t f = 0; f < n_kf; ++f) {
        if (f > 0 && h_t_kf[f] < h_t_kf[f - 1])
            return fail(ctx, LSR_EINVAL, "keyframe time stamps must not decrease (keyframe %d)", f);
        for (int k = 0; k < 16; ++k)
            if (!std::isfinite(h_T_old[16 * f + k]) || !std::isfinite(h_T_new[16 * f + k]))
                return fail(ctx, LSR_EINVAL, "non-finite pose of keyframe %d", f);
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        HIPCHK(ctx, fill<int64_t>(d_n_kept, 0, 1, s));
        return LSR_OK;
    }
    std::vector<char> key;
    put(key, (int)K_SURFEL);
    put(key, n);
    put(key, n_kf);
    for (int a = 0; a < 6; ++a) put(key, out[a]);
    Plan *pl = find_plan(ctx, key);
    int rc;
    if (!pl) {
        auto P = std::make_unique<Plan>();
        P->key = key;
        if (capturing(s)) return fail(ctx, LSR_ENOMEM, "allocation during capture");
        if ((rc = plan_malloc(ctx, P.get(), surfel_ws_bytes(n, n_kf)))) return rc;
        HIPCHK(ctx, hipHostMalloc((void **)&P->hmem, 64, hipHostMallocDefault));
        std::memcpy(P->hmem, out, 6 * sizeof(float *));
        SurfelWs w = surfel_carve(P->dmem, n, n_kf);
        HIPCHK(ctx, hipMemcpyAsync(w.out_ptrs, P->hmem, 6 * sizeof(float *), hipMemcpyHostToDevice, s));
        if ((rc = add_plan(ctx, std::move(P), &pl))) return rc;
    }
    SurfelWs w = surfel_carve(pl->dmem, n, n_kf);
    if (n_kf > 0) {
        // stream-ordered copies that return once done: the host arrays may change after the call
        HIPCHK(ctx, hipMemcpyWithStream(w.T_old, h_T_old, sizeof(double) * 16 * n_kf, hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyWithStream(w.T_new, h_T_new, sizeof(double) * 16 * n_kf, hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyWithStream(w.t_kf, h_t_kf, sizeof(int32_t) * n_kf, hipMemcpyHostToDevice, s));
    }
    HIPCHK(ctx, launch_surfel_correct(surfels, d_t0, d_tu, n, w, n_kf, *cam, w.out_ptrs, d_new_index, d_k_obs,
                                      d_n_kept, s));
    return LSR_OK;
}

void lsr_default_loop_params(lsr_loop_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->lambda = 1000.0;
    p->tau = 0.2;
    p->l_min = 0.25;
    p->tol = 1e-12;
    p->eps = 0.05f;
    p->max_iter = 100;
}

static int check_edges(lsr_ctx *ctx, const lsr_edge *e, int32_t m, int32_t n_frags, const char *what) {
    if (m > 0 && !e) return fail(ctx, LSR_EINVAL, "%s: NULL edge array", what);
    for (int32_t k = 0; k < m; ++k) {
        if (e[k].i < 0 || e[k].j < 0 || e[k].i >= n_frags || e[k].j >= n_frags || e[k].i == e[k].j)
            return fail(ctx, LSR_EINVAL, "%s %d joins fragments %d and %d (of %d)", what, k, e[k].i, e[k].j, n_frags);
        for (int q = 0; q < 16; ++q)
            if (!std::isfinite(e[k].T[q])) return fail(ctx, LSR_EINVAL, "%s %d: non-finite transform", what, k);
    }
    return LSR_OK;
}

// Edge information of `edges` over a plan whose pair e is (frags[i_e], frags[j_e]).
static int edge_info_run(lsr_ctx *ctx, const lsr_cloud *frags, int32_t n_frags, const lsr_edge *edges,
                         int32_t m, float eps, double *d_info, int64_t *d_count, hipStream_t s) {
    int rc;
    std::vector<FragIn> fr;
    int64_t nblk = 0;
    for (int32_t k = 0; k < m; ++k) {
        const lsr_cloud *a = frags + edges[k].i, *b = frags + edges[k].j;
        fr.push_back(frag_of(a, 0, a->n));
        fr.push_back(frag_of(b, 0, b->n));
        nblk += (a->n + 255) / 256 + (b->n + 255) / 256;
    }
    std::vector<char> key;
    put(key, (int)K_EDGE);
    put(key, m);
    for (auto &f : fr) put(key, f);
    const size_t a_bytes = sizeof(double) * 16 * (size_t)m, part_bytes = sizeof(double) * 10 * (size_t)(nblk + 1);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, nullptr, key, s, &pl, a_bytes + part_bytes + 512))) return rc;
    double *dA = (double *)pl->extra;
    double *partial = (double *)((char *)pl->extra + ((a_bytes + 255) & ~(size_t)255));
    std::vector<double> A(16 * (size_t)m);
    for (int32_t k = 0; k < m; ++k) std::memcpy(&A[16 * (size_t)k], edges[k].T, sizeof(double) * 16);
    if (m > 0) HIPCHK(ctx, hipMemcpyWithStream(dA, A.data(), a_bytes, hipMemcpyHostToDevice, s));
    tmark("edge_start", s);
    HIPCHK(ctx, build_grids(pl->g, eps, s));
    tmark("edge_grids", s);
    HIPCHK(ctx, launch_edge_info(pl->g, dA, m, eps, partial, d_info, d_count, s));
    tmark("edge_info", s);
    return LSR_OK;
}

static int check_frags(lsr_ctx *ctx, const lsr_cloud *frags, int32_t n_frags) {
    if (!frags || n_frags < 1) return fail(ctx, LSR_EINVAL, "no fragments");
    int rc;
    for (int32_t f = 0; f < n_frags; ++f)
        if ((rc = check_cloud(ctx, frags + f, "fragment", false))) return rc;
    return LSR_OK;
}

int lsr_edge_info(lsr_ctx *ctx, const lsr_cloud *frags, int32_t n_frags, const lsr_edge *h_edges,
                  int32_t n_edges, float eps, double *d_info, int64_t *d_count, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_frags(ctx, frags, n_frags)) || (rc = check_edges(ctx, h_edges, n_edges, n_frags, "edge")))
        return rc;
    if (n_edges < 0 || !(eps > 0) || !(eps < 1e30f) || (n_edges > 0 && (!d_info || !d_count)))
        return fail(ctx, LSR_EINVAL, "bad edge-information arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (n_edges == 0) return LSR_OK;
    return edge_info_run(ctx, frags, n_frags, h_edges, n_edges, eps, d_info, d_count, (hipStream_t)stream);
}

static int check_loop_params(lsr_ctx *ctx, const lsr_loop_params *p) {
    if (!p) return fail(ctx, LSR_EINVAL, "NULL loop parameters");
    if (!(p->lambda > 0) || !std::isfinite(p->lambda) || !(p->tau > 0) || !std::isfinite(p->tau) ||
        !(p->l_min >= 0) || !(p->l_min <= 1) || !(p->tol >= 0) || !std::isfinite(p->tol) || !(p->eps > 0) ||
        !(p->eps < 1e30f) || p->max_iter < 0)
        return fail(ctx, LSR_EINVAL, "bad loop parameters");
    return LSR_OK;
}

// Plan of a pose-graph solve: device copies of the poses and edges, per-candidate scratch.
static int loop_solve_run(lsr_ctx *ctx, int32_t n, const double *h_T_init, const lsr_edge *h_odo,
                          const double *d_info_odo, const lsr_edge *h_loops, int32_t n_loops,
                          const double *d_info_loop, const int64_t *d_count_loop, const lsr_loop_params *prm,
                          double *d_T_out, lsr_loop_result *d_res, hipStream_t s) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bT = al(sizeof(double) * 16 * (size_t)n), bo = al(sizeof(lsr_edge) * (size_t)(n - 1)),
                 bl = al(sizeof(lsr_edge) * (size_t)std::max(n_loops, 1)),
                 bs = al(loop_scratch_bytes(n, std::max(n_loops, 1)));
    std::vector<char> key;
    put(key, (int)K_LOOP);
    put(key, n);
    put(key, n_loops);
    Plan *pl = find_plan(ctx, key);
    int rc;
    if (!pl) {
        auto P = std::make_unique<Plan>();
        P->key = key;
        if (capturing(s)) return fail(ctx, LSR_ENOMEM, "allocation during capture");
        if ((rc = plan_malloc(ctx, P.get(), bT + bo + bl + bs))) return rc;
        if ((rc = add_plan(ctx, std::move(P), &pl))) return rc;
    }
    double *dT = (double *)pl->dmem;
    lsr_edge *dodo = (lsr_edge *)(pl->dmem + bT);
    lsr_edge *dloops = (lsr_edge *)(pl->dmem + bT + bo);
    double *scratch = (double *)(pl->dmem + bT + bo + bl);
    HIPCHK(ctx, hipMemcpyWithStream(dT, h_T_init, sizeof(double) * 16 * (size_t)n, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyWithStream(dodo, h_odo, sizeof(lsr_edge) * (size_t)(n - 1), hipMemcpyHostToDevice, s));
    if (n_loops > 0)
        HIPCHK(ctx, hipMemcpyWithStream(dloops, h_loops, sizeof(lsr_edge) * (size_t)n_loops, hipMemcpyHostToDevice,
                                        s));
    tmark("loop_start", s);
    HIPCHK(ctx, launch_loop_solve(n, dT, dodo, d_info_odo, dloops, n_loops, d_info_loop, d_count_loop, *prm,
                                  scratch, d_T_out, d_res, s));
    tmark("loop_solve", s);
    return LSR_OK;
}

static int check_chain(lsr_ctx *ctx, int32_t n, const double *h_T_init, const lsr_edge *h_odo, const lsr_edge *h_loops,
                       int32_t n_loops) {
    if (n < 2 || n > 4096) return fail(ctx, LSR_EINVAL, "chain of %d nodes (2 .. 4096)", n);
    if (n_loops < 0) return fail(ctx, LSR_EINVAL, "negative loop count");
    if (!h_T_init) return fail(ctx, LSR_EINVAL, "NULL initial poses");
    for (int64_t k = 0; k < 16 * (int64_t)n; ++k)
        if (!std::isfinite(h_T_init[k])) return fail(ctx, LSR_EINVAL, "non-finite initial pose");
    int rc;
    if ((rc = check_edges(ctx, h_odo, n - 1, n, "odometry edge")) ||
        (rc = check_edges(ctx, h_loops, n_loops, n, "loop candidate")))
        return rc;
    for (int32_t k = 0; k < n - 1; ++k)
        if (std::min(h_odo[k].i, h_odo[k].j) != k || std::max(h_odo[k].i, h_odo[k].j) != k + 1)
            return fail(ctx, LSR_EINVAL, "odometry edge %d must join nodes %d and %d", k, k, k + 1);
    return LSR_OK;
}

int lsr_loop_solve(lsr_ctx *ctx, int32_t n_nodes, const double *h_T_init, const lsr_edge *h_odo,
                   const double *d_info_odo, const lsr_edge *h_loops, int32_t n_loops, const double *d_info_loop,
                   const int64_t *d_count_loop, const lsr_loop_params *prm, double *d_T_out,
                   lsr_loop_result *d_res, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_loop_params(ctx, prm)) || (rc = check_chain(ctx, n_nodes, h_T_init, h_odo, h_loops, n_loops)))
        return rc;
    if (!d_info_odo || (n_loops > 0 && (!d_info_loop || !d_count_loop || !d_res)))
        return fail(ctx, LSR_EINVAL, "NULL loop-solve array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return loop_solve_run(ctx, n_nodes, h_T_init, h_odo, d_info_odo, h_loops, n_loops, d_info_loop, d_count_loop,
                          prm, d_T_out, d_res, (hipStream_t)stream);
}

int lsr_loop_verify(lsr_ctx *ctx, const lsr_cloud *frags, int32_t n_frags, const double *h_T_init,
                    const lsr_edge *h_odo, const lsr_edge *h_loops, int32_t n_loops, const lsr_loop_params *prm,
                    double *d_T_out, lsr_loop_result *d_res, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_loop_params(ctx, prm)) || (rc = check_frags(ctx, frags, n_frags)) ||
        (rc = check_chain(ctx, n_frags, h_T_init, h_odo, h_loops, n_loops)))
        return rc;
    if (n_loops > 0 && !d_res) return fail(ctx, LSR_EINVAL, "NULL loop results");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int32_t m = n_frags - 1 + n_loops;
    std::vector<lsr_edge> all(h_odo, h_odo + (n_frags - 1));
    all.insert(all.end(), h_loops, h_loops + n_loops);
    // information and counts of every edge: a plan of its own keyed by the chain's size
    std::vector<char> key;
    put(key, (int)K_LOOP);
    put(key, -1);
    put(key, m);
    Plan *pl = find_plan(ctx, key);
    if (!pl) {
        auto P = std::make_unique<Plan>();
        P->key = key;
        if (capturing(s)) return fail(ctx, LSR_ENOMEM, "allocation during capture");
        if ((rc = plan_malloc(ctx, P.get(), (sizeof(double) * 36 + sizeof(int64_t)) * (size_t)m + 256))) return rc;
        if ((rc = add_plan(ctx, std::move(P), &pl))) return rc;
    }
    double *info = (double *)pl->dmem;
    int64_t *cnt = (int64_t *)(pl->dmem + sizeof(double) * 36 * (size_t)m);
    pl->busy = true;             // the solve reads it after the next steps' allocations
    rc = edge_info_run(ctx, frags, n_frags, all.data(), m, prm->eps, info, cnt, s);
    if (!rc)
        rc = loop_solve_run(ctx, n_frags, h_T_init, h_odo, info, h_loops, n_loops, info + 36 * (size_t)(n_frags - 1),
                            cnt + (n_frags - 1), prm, d_T_out, d_res, s);
    pl->busy = false;
    return rc;
}

static int64_t ransac_hyp_count(int64_t n_hyp, int64_t nP) {
    return n_hyp > 0 ? n_hyp : std::min<int64_t>(4000000, 100 * nP);
}

int lsr_ransac_pair(lsr_ctx *ctx, const lsr_cloud *P, const lsr_cloud *Q, const lsr_params *prm, int64_t n_hyp,
                    lsr_ransac_result *d_out, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_params(ctx, prm)) || (rc = check_cloud(ctx, P, "P", true)) || (rc = check_cloud(ctx, Q, "Q", true)))
        return rc;
    if (!d_out) return fail(ctx, LSR_EINVAL, "d_out is NULL");
    if (n_hyp > ((int64_t)1 << 31) - 1) return fail(ctx, LSR_EINVAL, "n_hyp %lld too large", (long long)n_hyp);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nh = ransac_hyp_count(n_hyp, P->n);
    std::vector<FragIn> fr = {frag_of(P, 0, P->n), frag_of(Q, 0, Q->n)};
    std::vector<char> key;
    put(key, (int)K_RANSAC);
    put(key, *prm);
    put(key, nh);
    for (auto &f : fr) { put(key, f.n); for (int a = 0; a < 6; ++a) put(key, f.src[a]); }
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, prm, key, s, &pl, ransac_bytes(nh)))) return rc;
    const float r_cell = std::max(std::max(prm->r_normal, prm->r_feature), prm->max_corr);
    HIPCHK(ctx, fill<uint32_t>((uint32_t *)pl->ps, 0u, (int64_t)(sizeof(PairState) / 4), s));
    HIPCHK(ctx, build_grids(pl->g, r_cell, s));
    HIPCHK(ctx, launch_normals(pl->g, prm->r_normal, pl->d, nullptr, s));
    HIPCHK(ctx, launch_spfh(pl->g, prm->r_feature, pl->d, s));
    HIPCHK(ctx, launch_fpfh(pl->g, prm->r_feature, pl->d, pl->ps, s));
    if (prm->precision == LSR_BF16_SCREEN)
        HIPCHK(ctx, launch_match_bf16(pl->g, pl->d, pl->m, pl->ps, pl->mscratch, ctx->tune_screen, s));
    else
        HIPCHK(ctx, launch_match_fp32(pl->g, pl->d, pl->m, s));
    tmark("match", s);
    HIPCHK(ctx, launch_ransac(pl->g, pl->d, pl->m, pl->ps, ransac_carve(pl->extra, nh), nh, *prm, pl->scan_tmp, d_out,
                              nullptr, s));
    tmark("ransac", s);
    return LSR_OK;
}

int lsr_stage_ransac(lsr_ctx *ctx, const lsr_cloud *P, const double *d_nrmP, const lsr_cloud *Q,
                     const double *d_nrmQ, const int32_t *d_nnQ, int64_t n_hyp, const lsr_params *prm,
                     lsr_ransac_result *d_out, const lsr_ransac_trace *tr, void *stream) {
    if (!ctx) return LSR_EINVAL;
    int rc;
    if ((rc = check_params(ctx, prm)) || (rc = check_cloud(ctx, P, "P", false)) || (rc = check_cloud(ctx, Q, "Q", false)))
        return rc;
    if (!d_out || (P->n > 0 && !d_nnQ) || (prm->normal_check && (!d_nrmP || !d_nrmQ)))
        return fail(ctx, LSR_EINVAL, "bad ransac arguments");
    if (n_hyp > ((int64_t)1 << 31) - 1) return fail(ctx, LSR_EINVAL, "n_hyp %lld too large", (long long)n_hyp);
    if (tr && tr->capacity < 0) return fail(ctx, LSR_EINVAL, "negative trace capacity");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nh = ransac_hyp_count(n_hyp, P->n);
    std::vector<FragIn> fr = {frag_of(P, 0, P->n), frag_of(Q, 0, Q->n)};
    std::vector<char> key;
    put(key, (int)K_RANSAC_STAGE);
    put(key, nh);
    for (auto &f : fr) put(key, f);
    Plan *pl = find_plan(ctx, key);
    if (!pl && (rc = make_batch_plan(ctx, fr, true, nullptr, key, s, &pl, ransac_bytes(nh)))) return rc;
    HIPCHK(ctx, fill<uint32_t>((uint32_t *)pl->ps, 0u, (int64_t)(sizeof(PairState) / 4), s));
    HIPCHK(ctx, build_grids(pl->g, prm->max_corr, s));
    if (prm->normal_check) {
        HIPCHK(ctx, copy<double>(pl->nrm_orig, d_nrmP, 3 * P->n, s));
        HIPCHK(ctx, copy<double>(pl->nrm_orig + 3 * P->n, d_nrmQ, 3 * Q->n, s));
        HIPCHK(ctx, launch_normals_inject(pl->g, pl->nrm_orig, pl->d, s));
    }
    HIPCHK(ctx, copy<int32_t>(pl->m.nn, d_nnQ, P->n, s));
    HIPCHK(ctx, launch_ransac(pl->g, pl->d, pl->m, pl->ps, ransac_carve(pl->extra, nh), nh, *prm, pl->scan_tmp, d_out,
                              tr, s));
    return LSR_OK;
}

static int align_common(lsr_ctx *ctx, bool bwd, const float *const P_xyz[3], int64_t nP,
                        const float *const Q_xyz[3], int64_t nQ,
                        const int32_t *d_corr, const int64_t *coff, int32_t n_problems, const double *d_T,
                        const double *d_mu, const double *d_dE, double *out, float *const dP[3], float *const dQ[3],
                        void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (nP < 0 || nQ < 0 || !P_xyz || !Q_xyz || !coff || n_problems <= 0 || n_problems > (1 << 20) || !d_T || !d_mu || !out)
        return fail(ctx, LSR_EINVAL, "bad align-loss arguments");
    for (int a = 0; a < 3; ++a)
        if (!P_xyz[a] || !Q_xyz[a] || (bwd && (!dP || !dQ || !dP[a] || !dQ[a])))
            return fail(ctx, LSR_EINVAL, "NULL coordinate or gradient array");
    if (bwd && !d_dE) return fail(ctx, LSR_EINVAL, "NULL dE");
    for (int k = 0; k < n_problems; ++k)
        if (coff[k] < 0 || coff[k + 1] < coff[k]) return fail(ctx, LSR_EINVAL, "bad correspondence offsets");
    if (coff[n_problems] > 0 && !d_corr) return fail(ctx, LSR_EINVAL, "NULL correspondences");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (nP >= INT32_MAX || nQ >= INT32_MAX || coff[n_problems] >= INT32_MAX)
        return fail(ctx, LSR_EINVAL, "align-loss sizes beyond 2^31 - 1");
    std::vector<char> key;
    put(key, (int)K_ALIGN);
    put(key, n_problems);
    put(key, bwd ? nP : (int64_t)-1);
    put(key, bwd ? nQ : (int64_t)-1);
    key.insert(key.end(), (const char *)coff, (const char *)(coff + n_problems + 1));
    Plan *pl = find_plan(ctx, key);
    if (!pl) {
        auto P = std::make_unique<Plan>();
        P->key = key;
        std::vector<int64_t> pblk(n_problems + 1);
        int64_t nb = align_blocks(coff, n_problems, nullptr, pblk.data());
        std::vector<char> tab(align_block_bytes() * (size_t)std::max<int64_t>(nb, 1));
        align_blocks(coff, n_problems, tab.data(), pblk.data());
        Layout H;
        size_t h_tab = H.add(tab.size()), h_pb = H.add(sizeof(int64_t) * pblk.size());
        Layout D;
        size_t o_tabs = D.add(H.total), o_part = D.add(sizeof(double) * 6 * (size_t)std::max<int64_t>(nb, 1));
        size_t o_seg = D.add(bwd ? align_seg_bytes(coff[n_problems], nP, nQ) : 256);
        if (capturing(s)) return fail(ctx, LSR_ENOMEM, "allocation during capture");
        HIPCHK(ctx, hipHostMalloc((void **)&P->hmem, H.total, hipHostMallocDefault));
        int rc1 = plan_malloc(ctx, P.get(), D.total);
        if (rc1) return rc1;
        std::memcpy(P->hmem + h_tab, tab.data(), tab.size());
        std::memcpy(P->hmem + h_pb, pblk.data(), sizeof(int64_t) * pblk.size());
        P->atab = P->dmem + o_tabs + h_tab;
        P->apblk = (int64_t *)(P->dmem + o_tabs + h_pb);
        P->apart = (double *)(P->dmem + o_part);
        P->extra = P->dmem + o_seg;
        P->anblk = nb;
        HIPCHK(ctx, hipMemcpyAsync(P->dmem + o_tabs, P->hmem, H.total, hipMemcpyHostToDevice, s));
        int rc;
        if ((rc = add_plan(ctx, std::move(P), &pl))) return rc;
    }
    HIPCHK(ctx, launch_align(bwd, P_xyz, nP, Q_xyz, nQ, d_corr, coff[n_problems], pl->atab, pl->anblk, pl->apblk,
                             n_problems, d_T, d_mu, d_dE, pl->apart, out, dP, dQ, (char *)pl->extra, s));
    return LSR_OK;
}

int lsr_align_loss(lsr_ctx *ctx, const float *const P_xyz[3], int64_t nP, const float *const Q_xyz[3], int64_t nQ,
                   const int32_t *d_corr, const int64_t *coff, int32_t n_problems, const double *d_T,
                   const double *d_mu, double *d_E, void *stream) {
    return align_common(ctx, false, P_xyz, nP, Q_xyz, nQ, d_corr, coff, n_problems, d_T, d_mu, nullptr, d_E, nullptr,
                        nullptr, stream);
}

int lsr_align_loss_backward(lsr_ctx *ctx, const float *const P_xyz[3], int64_t nP,
                            const float *const Q_xyz[3], int64_t nQ, const int32_t *d_corr, const int64_t *coff, int32_t n_problems, const double *d_T,
                            const double *d_mu, const double *d_dE, float *const dP_xyz[3], float *const dQ_xyz[3],
                            double *d_dxi, void *stream) {
    if (!d_dxi) return ctx ? fail(ctx, LSR_EINVAL, "NULL d_dxi") : LSR_EINVAL;
    return align_common(ctx, true, P_xyz, nP, Q_xyz, nQ, d_corr, coff, n_problems, d_T, d_mu, d_dE, d_dxi, dP_xyz, dQ_xyz,
                        stream);
}

int lsr_se3_retract(lsr_ctx *ctx, int32_t n, const double *d_xi, const double *d_T, double *d_T_out, void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (n < 0 || (n > 0 && (!d_xi || !d_T || !d_T_out))) return fail(ctx, LSR_EINVAL, "bad retraction arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_retract(n, d_xi, d_T, d_T_out, (hipStream_t)stream));
    return LSR_OK;
}

int lsr_se3_retract_grad(lsr_ctx *ctx, int32_t n, const double *d_xi, const double *d_g_left, double *d_g_xi,
                         void *stream) {
    if (!ctx) return LSR_EINVAL;
    if (n < 0 || (n > 0 && (!d_xi || !d_g_left || !d_g_xi))) return fail(ctx, LSR_EINVAL, "bad retraction arguments");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_retract_grad(n, d_xi, d_g_left, d_g_xi, (hipStream_t)stream));
    return LSR_OK;
}

}  // extern "C"
