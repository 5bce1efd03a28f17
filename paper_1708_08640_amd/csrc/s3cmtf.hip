// Host side of the C ABI declared in include/s3cmtf.h.
//
// Every device buffer is the caller's; the plan carves its working arrays
// out of one caller-provided workspace (bump allocation, 256-byte aligned).
#include "s3cmtf.h"


#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace s3;

namespace {

s3_status fail(s3_plan *p, s3_status st, const char *fmt, ...) {
    if (p) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        p->err = buf;
    }
    return st;
}

#define HIPCHK(plan, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(plan, S3_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

bool pick_set_any(bool f64, int N, int JP, KernelSet *ks, bool naive, bool cp, bool matrix, bool bf16) {
    if (matrix) return !f64 && pick_mx(bf16, N, JP, ks);
    if (cp) return pick_cp(f64, N, JP, ks);
    if (naive) return pick_naive(f64, N, JP, ks);
    if (f64) return pick_reuse_f64(N, JP, ks);
    return N == 3 ? pick_reuse_f32_3(JP, ks) : pick_reuse_f32_4(JP, ks);
}

int padded_rank(int N, int Jmax) {
    static const int p3[] = {3, 4, 8, 10, 12, 16};
    static const int p4[] = {2, 4, 8};
    if (N == 3) {
        for (int v : p3) if (Jmax <= v) return v;
    } else if (N == 4) {
        for (int v : p4) if (Jmax <= v) return v;
    }
    return 0;
}

// profiling event k (created on first use): the pairs 2i, 2i + 1 take the
// start and end of the i-th dominant-kernel dispatch of an epoch, stamped by
// the dispatch itself (hipExtLaunchKernelGGL), so they time the kernel alone.
// They are timing-only events without the system-scope fence, whose cache
// write-back would otherwise land in the timed interval and slow the next
// kernel; the epoch's end event, waited on before they are read, has it.
hipEvent_t prof_event(s3_plan *p, size_t k) {
    while (p->pev.size() <= k) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        p->pev.push_back(e);
    }
    return p->pev[k];
}

double eta_of(const s3_desc &d, int epoch) { return d.eta0 / (1.0 + d.mu * (double)epoch); }

// launch helper for the row-apply kernel (J <= 16)
// the batch's row updates of every group: one reduce launch, and one finish
// launch when some row has more than kLongSeg contributions
template <typename T>
void rows_apply(s3_plan *p, int64_t b, void *const *P, double eta, double kappa, int damp, int acc,
                const CoreStep<T> *core, hipStream_t st) {
    RowsArgs<T> a{};
    a.G = p->N + p->M;
    a.scr = (const T *)p->scr;
    a.part = (T *)p->rows_part;
    a.eta = (T)eta;
    a.kappa = (T)kappa;
    a.damp = damp;
    a.accumulate = acc;
    int64_t blk = 0, pieces = 0;
    for (int gi = 0; gi < a.G; ++gi) {
        const Group &G = p->grp[gi];
        RowsGroup &r = a.g[gi];
        r.contrib = G.contrib;
        r.seg_start = G.seg_start;
        r.seg_row = G.seg_row;
        r.med_ids = G.med_ids;
        r.long_ids = G.long_ids;
        r.long_fp = G.long_fp;
        r.pc0 = G.pc0;
        r.pc1 = G.pc1;
        r.P = P[gi];
        r.J = G.J;
        const bool any = G.nseg > 0;
        r.s0 = any ? G.h_boff[b] : 0;
        r.s1 = any ? G.h_boff[b + 1] : 0;
        r.m0 = any ? G.h_moff[b] : 0;
        r.m1 = any ? G.h_moff[b + 1] : 0;
        r.l0 = any ? G.h_loff[b] : 0;
        r.l1 = any ? G.h_loff[b + 1] : 0;
        r.p0 = any ? G.h_poff[b] : 0;
        r.p1 = any ? G.h_poff[b + 1] : 0;
        r.b_lane = blk;
        blk += (r.s1 - r.s0 + kRowsThreads - 1) / kRowsThreads;
        r.b_med = blk;
        blk += (r.m1 - r.m0 + kRowsThreads / kWave - 1) / (kRowsThreads / kWave);
        r.b_piece = blk;
        blk += r.p1 - r.p0;
        a.part_base[gi] = pieces;
        pieces += r.p1 - r.p0;
        a.n_long += r.l1 - r.l0;
    }
    a.b_end = blk;
    if (core) {
        a.core = *core;
        blk += core->blocks;
    }
    if (blk > 0) hipLaunchKernelGGL(k_rows_reduce<T>, dim3((unsigned)blk), dim3(kRowsThreads), 0, st, a);
    if (a.n_long > 0)
        hipLaunchKernelGGL(k_rows_finish<T>, dim3((unsigned)((a.n_long * kWave + kRowsThreads - 1) / kRowsThreads)),
                           dim3(kRowsThreads), 0, st, a);
}

// the core step of a batch of nt tensor entries (run by k_rows_reduce)
template <typename T> CoreStep<T> core_step(s3_plan *p, int64_t nt, double eta, bool acc, void *dst) {
    CoreStep<T> c{};
    c.G = (T *)dst;
    c.Gp = acc ? nullptr : (T *)p->Gp;
    c.part = (const T *)p->part;
    c.part_curv = (const T *)p->part_curv;
    c.nchunks = (nt + p->ks.det_chunk - 1) / p->ks.det_chunk;
    c.nt = nt;
    c.KP = p->KP;
    c.blocks = (p->KP + 15) / 16;
    c.Nc = p->d.core_kind == S3_CORE_CP ? 1 : p->N;
    c.JP = p->JP;
    for (int n = 0; n < kMaxN; ++n) c.Js[n] = n < p->N ? p->d.rank[n] : 1;
    c.reg_core = (T)(p->d.lambda_reg / (double)p->nX);
    c.eta = (T)eta;
    c.kappa = (T)(p->N + 1);
    c.damp = p->d.damping;
    c.accumulate = acc ? 1 : 0;
    return c;
}

template <typename T> void pad_core(s3_plan *p, hipStream_t st, void *dst = nullptr) {
    const int *J = p->d.rank;
    // a hyper-diagonal core pads as a one-mode core of J values
    const int Nc = p->d.core_kind == S3_CORE_CP ? 1 : p->N;
    hipLaunchKernelGGL(k_pad_core<T>, dim3(grid_for(p->KP, 256, 64)), dim3(256), 0, st, (const T *)p->b.G,
                       (T *)(dst ? dst : p->Gp), Nc, p->JP, J[0], J[1], J[2], p->N > 3 ? J[3] : 1);
}

template <typename T> void fill(void *ptr, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, (T *)ptr, n, (T)v);
}

// One det-mode batch.  gx/gy non-null: adjoint pass (accumulate into
// dU/dG/dV).  Launches: the batch's entries (and, except for an FP64 Tucker
// core, its chunk core partials), then the row sums with the core step in the
// same launch, then the longest rows' pieces.  The padded core copy Gp must
// be current on entry; the training core step keeps it so.
template <typename T>
void det_batch(s3_plan *p, int64_t b, double eta, const void *gx, const void *const *gy, void *const *dU,
               void *dG, void *const *dV, hipStream_t st) {
    const int M = p->M;
    const bool adj = (gx != nullptr) || (gy != nullptr) || (dG != nullptr);
    const int64_t *to = p->h_type_off.data() + b * (M + 1);
    const int64_t t0 = to[0], nt = to[1] - to[0];
    // the adjoint without a tensor (or a matrix) sensitivity contributes zeros
    const bool t_zero = adj && gx == nullptr;
    if (nt > 0 && t_zero) fill<T>(p->scr, nt * p->t_stride, 0.0, st);
    DetMatArgs<T> B{};
    B.M = M;
    B.lambda_m = (T)p->d.lambda_m;
    B.lambda_reg = (T)p->d.lambda_reg;
    const int64_t t_blocks = (nt > 0 && !t_zero) ? (nt + p->ks.det_chunk - 1) / p->ks.det_chunk : 0;
    int64_t blocks = t_blocks;
    for (int m = 0; m < M; ++m) {
        const int64_t m0 = to[m + 1], nm = to[m + 2] - to[m + 1];
        T *scr = (T *)p->scr + p->m_base[m];
        const int c = p->d.mat_mode[m];
        DetMatrix<T> &d = B.m[m];
        d.b0 = blocks;
        if (nm <= 0) continue;
        if (adj && (gy == nullptr || gy[m] == nullptr)) {
            fill<T>(scr, nm * p->m_stride[m], 0.0, st);
            continue;
        }
        d.ids = p->sorted_ids + m0;
        d.n = nm;
        d.id_base = p->mat_begin[m];
        d.row = p->bidx + m0;                // item order
        d.col = p->bidx + p->n_items + m0;
        d.val = (const T *)p->bval + m0;
        d.Uc = (const T *)p->b.U[c];
        d.V = (const T *)p->b.V[m];
        d.cntV = p->cntV[m];
        d.gy = adj ? (const T *)gy[m] : nullptr;
        d.scr = scr;
        d.J = p->d.rank[c];
        blocks += (nm + kChunk - 1) / kChunk;
    }
    if (blocks > 0) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (p->prof && !adj) {
            e0 = prof_event(p, p->pev_used);
            e1 = prof_event(p, p->pev_used + 1);
            if (e0 && e1) p->pev_used += 2;
            else e0 = e1 = nullptr;
        }
        if (t_blocks > 0) p->ks.mx_format(p, st);  // the core as the last batch left it
        p->ks.det_entries(p, p->sorted_ids + t0, nt, t_blocks, adj ? gx : nullptr, &B, blocks, st, e0, e1);
    }
    if (t_blocks > 0) p->ks.core_partial(p, p->sorted_ids + t0, nt, st);
    void *P[S3_MAX_ORDER + S3_MAX_MATRICES];
    for (int g = 0; g < p->N + M; ++g)
        P[g] = (g < p->N) ? (adj ? dU[g] : p->b.U[g]) : (adj ? dV[g - p->N] : p->b.V[g - p->N]);
    const CoreStep<T> core = core_step<T>(p, nt, eta, adj, adj ? dG : p->b.G);
    rows_apply<T>(p, b, P, eta, (double)(p->N + 1), p->d.damping, adj ? 1 : 0, t_blocks > 0 ? &core : nullptr, st);
}

template <typename T> size_t layout(s3_plan *p, void *base, int64_t x_nnz, int64_t t_nnz,
                                    const int64_t *y_nnz, bool with_order, size_t *temp_bytes_out);

// The det-mode build packs each contribution's per-batch scratch offsets into
// 32-bit halves and sorts items by a 32-bit (batch, type) key: both must fit.
bool det_fits_32bit(const s3_plan *p, int64_t x_nnz, const int64_t *y_nnz) {
    const int N = p->N, M = p->M;
    const int64_t B = p->d.batch;
    int64_t n_items = x_nnz;
    for (int m = 0; m < M; ++m) n_items += y_nnz[m];
    const int64_t nb = (n_items + B - 1) / B;
    int64_t end = std::min(B, x_nnz) * ((int64_t)N * p->JP + N + 2);  // as the per-batch scratch carve
    for (int m = 0; m < M; ++m)
        end += std::min(B, std::max<int64_t>(y_nnz[m], 1)) * (2 * (int64_t)p->d.rank[p->d.mat_mode[m]] + 2);
    const int64_t lim = (int64_t)1 << 32;
    return end < lim && nb * (M + 1) <= lim;
}

}  // namespace

// ------------------------------------------------ allocation-free prediction

// Device memory of s3_predict_noalloc: one flag word for the index check (in
// the first 256 bytes), then the zero-padded core.  Each GPU the library runs
// on holds its own copy until the process ends.
constexpr size_t kStaticScratchBytes = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};  // per device: the address of its copy

// Address of `scratch` on the current device, looked up once per device with
// that device current.  (The array's name in host code is only a host-side
// handle; kernels must be given this address.)
s3_status scratch_ptr(s3_plan *p, void **out) {
    int dev = 0;
    HIPCHK(p, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(p, S3_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        HIPCHK(p, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(p, S3_ERR_HIP, "hipGetSymbolAddress gave a null address");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return S3_OK;
}

}  // namespace

// ========================================================================== ABI

extern "C" {

const char *s3_status_string(s3_status st) {
    switch (st) {
    case S3_OK: return "ok";
    case S3_ERR_INVALID_ARG: return "invalid argument";
    case S3_ERR_INDEX_RANGE: return "index out of range";
    case S3_ERR_UNSUPPORTED: return "unsupported configuration";
    case S3_ERR_NONFINITE: return "non-finite result";
    case S3_ERR_HIP: return "HIP runtime error";
    case S3_ERR_WORKSPACE: return "workspace too small";
    case S3_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

s3_status s3_last_error(const s3_plan *plan, char *buf, size_t len) {
    if (!plan || !buf || len == 0) return S3_ERR_INVALID_ARG;
    snprintf(buf, len, "%s", plan->err.c_str());
    return S3_OK;
}

s3_status s3_plan_create(const s3_desc *desc, s3_plan **out) {
    if (!desc || !out) return S3_ERR_INVALID_ARG;
    *out = nullptr;
    const s3_desc &d = *desc;
    if (d.order < 3 || d.order > S3_MAX_ORDER) return S3_ERR_UNSUPPORTED;
    if (d.n_mat < 0 || d.n_mat > S3_MAX_MATRICES) return S3_ERR_INVALID_ARG;
    if (d.dtype != S3_F64 && d.dtype != S3_F32 && d.dtype != S3_BF16) return S3_ERR_UNSUPPORTED;
    if (d.damping != S3_DAMP_NONE && d.damping != S3_DAMP_CURVATURE) return S3_ERR_INVALID_ARG;
    if (d.batch < 1 || d.round_items < 1 || d.hot_rows < -1 || d.hot_rows > 256) return S3_ERR_INVALID_ARG;
    if (d.contraction != S3_CONTRACT_REUSE && d.contraction != S3_CONTRACT_NAIVE &&
        d.contraction != S3_CONTRACT_MATRIX)
        return S3_ERR_INVALID_ARG;
    // BF16 operands exist only on the matrix cores; the matrix cores take FP32 or BF16
    if (d.dtype == S3_BF16 && d.contraction != S3_CONTRACT_MATRIX) return S3_ERR_UNSUPPORTED;
    if (d.dtype == S3_F64 && d.contraction == S3_CONTRACT_MATRIX) return S3_ERR_UNSUPPORTED;
    if (d.core_kind != S3_CORE_TUCKER && d.core_kind != S3_CORE_CP) return S3_ERR_INVALID_ARG;
    if (d.core_kind == S3_CORE_CP) {
        for (int n = 1; n < d.order; ++n)
            if (d.rank[n] != d.rank[0]) return S3_ERR_INVALID_ARG;
        if (d.contraction != S3_CONTRACT_REUSE) return S3_ERR_UNSUPPORTED;
    }
    if (!(d.eta0 > 0) || !(d.mu >= 0) || !(d.lambda_reg >= 0) || !(d.lambda_m >= 0)) return S3_ERR_INVALID_ARG;
    int Jmax = 0;
    for (int n = 0; n < d.order; ++n) {
        if (d.dims[n] < 1 || d.dims[n] > INT32_MAX || d.rank[n] < 1) return S3_ERR_INVALID_ARG;
        Jmax = std::max(Jmax, (int)d.rank[n]);
    }
    for (int m = 0; m < d.n_mat; ++m) {
        if (d.mat_mode[m] < 0 || d.mat_mode[m] >= d.order) return S3_ERR_INVALID_ARG;
        if (d.mat_cols[m] < 1 || d.mat_cols[m] > INT32_MAX) return S3_ERR_INVALID_ARG;
    }
    const int JP = padded_rank(d.order, Jmax);
    if (JP == 0) return S3_ERR_UNSUPPORTED;
    s3_plan *p = new s3_plan();
    p->d = d;
    p->N = d.order;
    p->M = d.n_mat;
    p->JP = JP;
    if (d.core_kind == S3_CORE_CP) {
        p->K = d.rank[0];
        p->KP = JP;
    } else {
        for (int n = 0; n < p->N; ++n) { p->K *= d.rank[n]; p->KP *= JP; }
    }
    p->exact = true;
    for (int n = 0; n < p->N; ++n) p->exact = p->exact && d.rank[n] == JP;
    p->tsize = (d.dtype == S3_F64) ? 8 : 4;
    const bool naive = d.contraction == S3_CONTRACT_NAIVE;
    const bool cp = d.core_kind == S3_CORE_CP;
    const bool ok = pick_set_any(d.dtype == S3_F64, p->N, JP, &p->ks, naive, cp,
                                 d.contraction == S3_CONTRACT_MATRIX, d.dtype == S3_BF16);
    if (!ok) {
        delete p;
        return S3_ERR_UNSUPPORTED;
    }
    *out = p;
    return S3_OK;
}

s3_status s3_plan_destroy(s3_plan *p) {
    if (!p) return S3_ERR_INVALID_ARG;
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    for (hipEvent_t e : p->pev) (void)hipEventDestroy(e);
    delete p;
    return S3_OK;
}

s3_status s3_workspace_size(const s3_plan *cp, int64_t x_nnz, int64_t t_nnz, const int64_t *y_nnz,
                            size_t *bytes) {
    s3_plan *p = const_cast<s3_plan *>(cp);
    if (!p || !bytes || x_nnz < 1 || t_nnz < 0 || (p->M > 0 && !y_nnz)) return S3_ERR_INVALID_ARG;
    for (int m = 0; m < p->M; ++m)
        if (y_nnz[m] < 0) return S3_ERR_INVALID_ARG;
    if (!det_fits_32bit(p, x_nnz, y_nnz))
        return fail(p, S3_ERR_UNSUPPORTED, "det batches of %lld items: per-batch scratch offsets or batch keys "
                    "exceed 32 bits", (long long)p->d.batch);
    size_t temp = 0;
    s3_plan scratch_plan = *p;  // measuring carves null pointers: keep a bound plan's own intact
    *bytes = (p->tsize == 8) ? layout<double>(&scratch_plan, nullptr, x_nnz, t_nnz, y_nnz, true, &temp)
                             : layout<float>(&scratch_plan, nullptr, x_nnz, t_nnz, y_nnz, true, &temp);
    return S3_OK;
}

}  // extern "C"

namespace {

struct DetTemps {
    uint32_t *key_in, *key_out;
    int32_t *ids_in;
    int64_t *type_off;
    uint64_t *gk_in, *gk_out, *gv_in, *gv_out;
    int32_t *flags, *segid;
    uint32_t *segb;
    int64_t *boff;
    void *temp;
    size_t temp_bytes;
};

// bind-time temporaries of the det-mode build, carved identically for
// measuring and for use
void carve_det_temps(Carver &c, DetTemps &t, int64_t n, int64_t nb, int M) {
    t.key_in = c.take<uint32_t>((size_t)n);
    t.key_out = c.take<uint32_t>((size_t)n);
    t.ids_in = c.take<int32_t>((size_t)n);
    t.type_off = c.take<int64_t>((size_t)(nb * (M + 1) + 1));
    t.gk_in = c.take<uint64_t>((size_t)n);
    t.gk_out = c.take<uint64_t>((size_t)n);
    t.gv_in = c.take<uint64_t>((size_t)n);
    t.gv_out = c.take<uint64_t>((size_t)n);
    t.flags = c.take<int32_t>((size_t)n);
    t.segid = c.take<int32_t>((size_t)n);
    t.segb = c.take<uint32_t>((size_t)n);
    t.boff = c.take<int64_t>((size_t)nb + 1);
    t.temp_bytes = std::max(sort_temp_bytes(n), sizeof(int32_t) * scan_temp_elems(n));
    t.temp = c.take<char>(t.temp_bytes + 256);
}

// The det-mode structures (item order, reduction segments, per-batch
// scratch) and, after them, the temporaries that build them.
template <typename T>
void carve_det(s3_plan *p, Carver &c, int64_t x_nnz, const int64_t *y_nnz, size_t *temp_bytes_out) {
    const int N = p->N, M = p->M;
    int64_t n_items = x_nnz;
    for (int m = 0; m < M; ++m) n_items += y_nnz[m];
    const int64_t B = p->d.batch;
    const int64_t nb = (n_items + B - 1) / B;
    {
        p->sorted_ids = c.take<int32_t>((size_t)n_items);
        p->bidx = c.take<int32_t>((size_t)N * n_items);
        p->bval = c.take<T>((size_t)n_items);
        // groups
        for (int g = 0; g < N + M; ++g) {
            int64_t nv = 0;
            if (g < N) {
                nv = x_nnz;
                for (int m = 0; m < M; ++m)
                    if (p->d.mat_mode[m] == g) nv += y_nnz[m];
            } else {
                nv = y_nnz[g - N];
            }
            p->grp[g].n_valid = nv;
            p->grp[g].contrib = c.take<uint64_t>((size_t)std::max<int64_t>(nv, 1));
            p->grp[g].seg_start = c.take<int64_t>((size_t)nv + 1);
            p->grp[g].seg_row = c.take<int32_t>((size_t)std::max<int64_t>(nv, 1));
            p->grp[g].med_ids = c.take<int32_t>((size_t)(nv / kShortSeg + 1));
            p->grp[g].long_ids = c.take<int32_t>((size_t)(nv / kLongSeg + 1));
            p->grp[g].long_fp = c.take<int32_t>((size_t)(nv / kLongSeg + 2));
            p->grp[g].pc0 = c.take<int64_t>((size_t)(nv / kPiece + nv / kLongSeg + 2));
            p->grp[g].pc1 = c.take<int64_t>((size_t)(nv / kPiece + nv / kLongSeg + 2));
        }
        // per-batch scratch
        const int64_t RJ = (int64_t)N * p->JP;  // gradient rows at a fixed JP stride
        p->RJ = RJ;
        p->t_stride = RJ + N + 2;
        const int64_t max_nt = std::min(B, x_nnz);
        int64_t off = max_nt * p->t_stride;
        for (int m = 0; m < M; ++m) {
            const int Jc = p->d.rank[p->d.mat_mode[m]];
            p->m_stride[m] = 2 * Jc + 2;
            p->m_base[m] = off;
            off += std::min(B, std::max<int64_t>(y_nnz[m], 1)) * p->m_stride[m];
        }
        p->scr = c.take<T>((size_t)off);
        p->max_chunks = (max_nt + p->ks.det_chunk - 1) / p->ks.det_chunk;
        p->part = c.take<T>((size_t)(p->max_chunks * p->KP));
        p->part_curv = c.take<T>((size_t)p->max_chunks);
        // piece sums of one batch: every group's contributions in pieces,
        // plus one partial piece per long segment
        p->rows_part = c.take<T>((size_t)(N + M) * (B / kPiece + B / kLongSeg + 2) * (kRowsJ + 1));
        // bind-time temporaries (same carve as build_det, from an aligned start)
        c.off = (c.off + 255) & ~(size_t)255;
        const size_t t0 = c.off;
        DetTemps tmp;
        carve_det_temps(c, tmp, n_items, nb, M);
        if (temp_bytes_out) *temp_bytes_out = c.off - t0;
    }
}

// Carve the workspace.  Returns total bytes.  base == nullptr: measure only.
template <typename T>
size_t layout(s3_plan *p, void *base, int64_t x_nnz, int64_t t_nnz, const int64_t *y_nnz, bool with_order,
              size_t *temp_bytes_out) {
    Carver c(base);
    const int N = p->N, M = p->M;
    for (int n = 0; n < N; ++n) p->cnt[n] = c.take<int32_t>((size_t)p->d.dims[n]);
    for (int m = 0; m < M; ++m) p->cntV[m] = c.take<int32_t>((size_t)p->d.mat_cols[m]);
    p->Gp = c.take<T>((size_t)p->KP);
    p->mx_g = c.take<char>((size_t)32 * 1024);  // the largest matrix-core operand layout (FP32, 4,096 values x 2)
    p->flag = c.take<int32_t>(16);
    p->n_red = std::max<int64_t>({(int64_t)2 * kReduceBlocks, sq_blocks(x_nnz), sq_blocks(t_nnz)});
    p->red = c.take<double>((size_t)p->n_red);
    // lock-free structures
    lockfree_layout<T>(p->lf, c, N, M, p->d, x_nnz, y_nnz, p->KP, p->JP);
    // orthogonalisation
    p->qr_part = c.take<double>((size_t)kQrBlocks * kQrJ * kQrJ);
    p->qr_R = c.take<double>((size_t)N * 3 * kQrJ * kQrJ);
    p->qr_G = c.take<T>((size_t)p->K);
    p->det_carve_off = c.off;  // the det structures come last: an adjoint may carve them after bind
    if (with_order) carve_det<T>(p, c, x_nnz, y_nnz, temp_bytes_out);
    return c.off + 256;
}


template <typename T> s3_status build_det(s3_plan *p, char *tmp_base, hipStream_t st) {
    const int N = p->N, M = p->M;
    const int64_t n = p->n_items, B = p->d.batch;
    const int64_t nb = p->n_batches;
    Carver c(tmp_base);
    DetTemps t;
    carve_det_temps(c, t, n, nb, M);
    uint32_t *key_in = t.key_in, *key_out = t.key_out;
    int32_t *ids_in = t.ids_in;
    int64_t *type_off = t.type_off;
    uint64_t *gk_in = t.gk_in, *gk_out = t.gk_out, *gv_in = t.gv_in, *gv_out = t.gv_out;
    int32_t *flags = t.flags, *segid = t.segid;
    uint32_t *segb = t.segb;
    int64_t *boff = t.boff;
    void *temp = t.temp;

    int64_t mat_end[S3_MAX_MATRICES] = {};
    for (int m = 0; m < M; ++m) mat_end[m] = p->mat_begin[m] + p->y_nnz[m];
    int64_t *d_mat_end = (int64_t *)p->red;  // small staging (<= 4 values)
    HIPCHK(p, hipMemcpyAsync(d_mat_end, mat_end, sizeof(int64_t) * S3_MAX_MATRICES, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_order_keys, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p->b.order, n, B, p->nX,
                       (int32_t)M, (const int64_t *)d_mat_end, key_in, ids_in);
    const int64_t nkeys = nb * (M + 1);
    HIPCHK(p, radix_sort_pairs(key_in, ids_in, key_out, p->sorted_ids, n, bits_for((uint64_t)nkeys), temp, st));
    hipLaunchKernelGGL(k_bounds<uint32_t>, dim3(grid_for(n + 1, 256, 16384)), dim3(256), 0, st, key_out, n,
                       nkeys, type_off);
    {
        // indices and values in item order for the batch kernels
        GatherArgs<T> ga{};
        ga.ids = p->sorted_ids;
        ga.n = n;
        ga.nX = p->nX;
        ga.N = N;
        ga.M = M;
        ga.x_idx = p->b.x_idx;
        ga.x_val = (const T *)p->b.x_val;
        for (int m = 0; m < M; ++m) {
            ga.mat_begin[m] = p->mat_begin[m];
            ga.y_row[m] = p->b.y_row[m];
            ga.y_col[m] = p->b.y_col[m];
            ga.y_val[m] = (const T *)p->b.y_val[m];
        }
        ga.bidx = p->bidx;
        ga.bval = (T *)p->bval;
        hipLaunchKernelGGL(k_gather_items<T>, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, ga);
    }
    p->h_type_off.assign((size_t)nkeys + 1, 0);
    HIPCHK(p, hipMemcpyAsync(p->h_type_off.data(), type_off, sizeof(int64_t) * (nkeys + 1),
                             hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));

    GroupArgs ga{};
    ga.sorted_ids = p->sorted_ids;
    ga.sorted_keys = key_out;
    ga.type_off = type_off;
    ga.n = n;
    ga.M = M;
    ga.N = N;
    ga.nX = p->nX;
    ga.x_idx = p->b.x_idx;
    ga.x_nnz = p->nX;
    ga.t_stride = p->t_stride;
    ga.nb = nb;
    for (int m = 0; m < M; ++m) {
        ga.y_row[m] = p->b.y_row[m];
        ga.y_col[m] = p->b.y_col[m];
        ga.mat_begin[m] = p->mat_begin[m];
        ga.mat_mode[m] = p->d.mat_mode[m];
        ga.m_base[m] = p->m_base[m];
        ga.m_stride[m] = p->m_stride[m];
        ga.m_J[m] = p->d.rank[p->d.mat_mode[m]];
    }
    int64_t goff = 0;
    for (int g = 0; g < N + M; ++g) {
        Group &G = p->grp[g];
        ga.group = g;
        if (g < N) {
            ga.t_goff = goff;
            ga.t_coff = p->RJ + g;
            goff += p->JP;
            G.J = p->d.rank[g];
            G.rows = p->d.dims[g];
        } else {
            G.J = p->d.rank[p->d.mat_mode[g - N]];
            G.rows = p->d.mat_cols[g - N];
        }
        ga.rbits = bits_for((uint64_t)G.rows);
        hipLaunchKernelGGL(k_group_contrib, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, ga, gk_in, gv_in);
        HIPCHK(p, radix_sort_pairs(gk_in, gv_in, gk_out, gv_out, n, ga.rbits + bits_for((uint64_t)nb + 1), temp,
                                   st));
        const int64_t nv = G.n_valid;
        G.h_boff.assign((size_t)nb + 1, 0);
        G.h_moff.assign((size_t)nb + 1, 0);
        G.h_loff.assign((size_t)nb + 1, 0);
        G.h_poff.assign((size_t)nb + 1, 0);
        if (nv == 0) { G.nseg = 0; continue; }
        HIPCHK(p, hipMemcpyAsync(G.contrib, gv_out, sizeof(uint64_t) * nv, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_seg_flags, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, st, gk_out, nv, flags);
        HIPCHK(p, scan_i32(flags, segid, nv, false, (int32_t *)temp, st));
        hipLaunchKernelGGL(k_seg_write, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, st, gk_out, flags, segid,
                           nv, G.seg_start, G.seg_row, segb, ga.rbits);
        int32_t nseg32 = 0;
        HIPCHK(p, hipMemcpyAsync(&nseg32, segid + nv - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        G.nseg = nseg32;
        hipLaunchKernelGGL(k_bounds<uint32_t>, dim3(grid_for(G.nseg + 1, 256, 16384)), dim3(256), 0, st, segb,
                           G.nseg, nb, boff);
        HIPCHK(p, hipMemcpyAsync(G.h_boff.data(), boff, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        // medium and long segments per batch; the long ones cut into pieces
        G.h_moff.assign((size_t)nb + 1, 0);
        G.h_poff.assign((size_t)nb + 1, 0);
        if (G.nseg == 0) continue;
        uint32_t *lbatch = (uint32_t *)gk_in;  // free once this group's keys are sorted
        int64_t *lc0 = (int64_t *)gv_in;       // likewise
        auto list = [&](int64_t lo, int64_t hi, int32_t *ids, std::vector<int64_t> &h_off, bool bounds,
                        int64_t *count) -> s3_status {
            hipLaunchKernelGGL(k_seg_class, dim3(grid_for(G.nseg, 256, 16384)), dim3(256), 0, st, G.seg_start,
                               G.nseg, lo, hi, flags);
            HIPCHK(p, scan_i32(flags, segid, G.nseg, false, (int32_t *)temp, st));
            int32_t n32 = 0;
            HIPCHK(p, hipMemcpyAsync(&n32, segid + G.nseg - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            HIPCHK(p, hipStreamSynchronize(st));
            *count = n32;
            if (n32 == 0) return S3_OK;
            hipLaunchKernelGGL(k_seg_list, dim3(grid_for(G.nseg, 256, 16384)), dim3(256), 0, st, flags, segid,
                               G.nseg, segb, G.seg_start, ids, lbatch, bounds ? lc0 : (int64_t *)nullptr,
                               bounds ? lc0 + n32 : (int64_t *)nullptr);
            hipLaunchKernelGGL(k_bounds<uint32_t>, dim3(grid_for(n32 + 1, 256, 16384)), dim3(256), 0, st, lbatch,
                               (int64_t)n32, nb, boff);
            HIPCHK(p, hipMemcpyAsync(h_off.data(), boff, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, st));
            HIPCHK(p, hipStreamSynchronize(st));
            return S3_OK;
        };
        int64_t nmed = 0, nlong = 0;
        s3_status ls = list(kShortSeg, kLongSeg, G.med_ids, G.h_moff, false, &nmed);
        if (ls != S3_OK) return ls;
        ls = list(kLongSeg, INT64_MAX, G.long_ids, G.h_loff, true, &nlong);
        if (ls != S3_OK) return ls;
        if (nlong == 0) continue;
        std::vector<int64_t> c01((size_t)(2 * nlong));
        HIPCHK(p, hipMemcpyAsync(c01.data(), lc0, sizeof(int64_t) * 2 * nlong, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        std::vector<int32_t> fp((size_t)nlong + 1);
        std::vector<int64_t> q0, q1;
        for (int64_t i = 0; i < nlong; ++i) {
            fp[(size_t)i] = (int32_t)q0.size();
            for (int64_t c = c01[(size_t)i]; c < c01[(size_t)(nlong + i)]; c += kPiece) {
                q0.push_back(c);
                q1.push_back(std::min<int64_t>(c + kPiece, c01[(size_t)(nlong + i)]));
            }
        }
        fp[(size_t)nlong] = (int32_t)q0.size();
        for (int64_t bb = 0; bb <= nb; ++bb) G.h_poff[(size_t)bb] = fp[(size_t)G.h_loff[(size_t)bb]];
        HIPCHK(p, hipMemcpyAsync(G.long_fp, fp.data(), sizeof(int32_t) * fp.size(), hipMemcpyHostToDevice, st));
        HIPCHK(p, hipMemcpyAsync(G.pc0, q0.data(), sizeof(int64_t) * q0.size(), hipMemcpyHostToDevice, st));
        HIPCHK(p, hipMemcpyAsync(G.pc1, q1.data(), sizeof(int64_t) * q1.size(), hipMemcpyHostToDevice, st));
        HIPCHK(p, hipStreamSynchronize(st));
    }
    return S3_OK;
}

// The det structures from the storage order (training entries, then each
// matrix's entries), for an adjoint on a plan bound without an item order.
template <typename T> s3_status build_adjoint_order(s3_plan *p, hipStream_t st) {
    if (!det_fits_32bit(p, p->nX, p->y_nnz))
        return fail(p, S3_ERR_UNSUPPORTED, "adjoint batches of %lld items: per-batch scratch offsets or batch "
                    "keys exceed 32 bits", (long long)p->d.batch);
    size_t temp_bytes = 0;
    {
        s3_plan measure = *p;
        Carver c(nullptr);
        c.off = p->det_carve_off;
        carve_det<T>(&measure, c, p->nX, p->y_nnz, &temp_bytes);
        if (c.off + 256 > p->ws_bytes)
            return fail(p, S3_ERR_WORKSPACE, "the adjoint needs a workspace of %zu bytes, %zu bound",
                        c.off + 256, p->ws_bytes);
    }
    Carver c(p->ws_base);
    c.off = p->det_carve_off;
    carve_det<T>(p, c, p->nX, p->y_nnz, nullptr);
    char *tmp = (char *)p->ws_base + (c.off - temp_bytes);  // the temporaries close the carve
    const int32_t *saved = p->b.order;
    p->b.order = nullptr;
    s3_status s = build_det<T>(p, tmp, st);
    p->b.order = saved;
    if (s != S3_OK) return s;
    p->adj_ready = true;
    return S3_OK;
}

template <typename T> s3_status bind_impl(s3_plan *p, const s3_buffers *buf, void *ws, size_t ws_bytes,
                                          hipStream_t st) {
    const int N = p->N, M = p->M;
    int64_t y_nnz[S3_MAX_MATRICES] = {};
    for (int m = 0; m < M; ++m) y_nnz[m] = buf->y_nnz[m];
    const bool with_order = buf->order != nullptr;
    if (with_order && !det_fits_32bit(p, buf->x_nnz, y_nnz))
        return fail(p, S3_ERR_UNSUPPORTED, "det batches of %lld items: per-batch scratch offsets or batch keys "
                    "exceed 32 bits", (long long)p->d.batch);
    size_t temp_bytes = 0;
    const size_t need = layout<T>(p, nullptr, buf->x_nnz, buf->t_nnz, y_nnz, with_order, &temp_bytes);
    if (!ws || ws_bytes < need)
        return fail(p, S3_ERR_WORKSPACE, "workspace of %zu bytes given, %zu needed", ws_bytes, need);
    {
        // set-up of the allocation-free entry point's memory on this device
        void *sp = nullptr;
        s3_status s = scratch_ptr(p, &sp);
        if (s != S3_OK) return s;
    }
    p->b = *buf;
    p->ws_base = ws;
    p->ws_bytes = ws_bytes;
    p->nX = buf->x_nnz;
    p->nT = buf->t_nnz;
    int64_t n_items = p->nX;
    for (int m = 0; m < M; ++m) {
        p->y_nnz[m] = y_nnz[m];
        p->mat_begin[m] = n_items;
        n_items += y_nnz[m];
    }
    p->n_items = n_items;
    p->n_batches = (n_items + p->d.batch - 1) / p->d.batch;
    layout<T>(p, ws, buf->x_nnz, buf->t_nnz, y_nnz, with_order, nullptr);
    // index validation
    HIPCHK(p, hipMemsetAsync(p->flag, 0, sizeof(int32_t) * 16, st));
    for (int n = 0; n < N; ++n) {
        hipLaunchKernelGGL(k_check_range, dim3(grid_for(p->nX, 256, 4096)), dim3(256), 0, st,
                           buf->x_idx + (int64_t)n * p->nX, p->nX, p->d.dims[n], p->flag);
        if (p->nT > 0)
            hipLaunchKernelGGL(k_check_range, dim3(grid_for(p->nT, 256, 4096)), dim3(256), 0, st,
                               buf->t_idx + (int64_t)n * p->nT, p->nT, p->d.dims[n], p->flag);
    }
    for (int m = 0; m < M; ++m) {
        if (y_nnz[m] == 0) continue;
        hipLaunchKernelGGL(k_check_range, dim3(grid_for(y_nnz[m], 256, 4096)), dim3(256), 0, st, buf->y_row[m],
                           y_nnz[m], p->d.dims[p->d.mat_mode[m]], p->flag);
        hipLaunchKernelGGL(k_check_range, dim3(grid_for(y_nnz[m], 256, 4096)), dim3(256), 0, st, buf->y_col[m],
                           y_nnz[m], p->d.mat_cols[m], p->flag);
    }
    if (with_order)
        hipLaunchKernelGGL(k_check_range, dim3(grid_for(n_items, 256, 4096)), dim3(256), 0, st, buf->order,
                           n_items, n_items, p->flag + 1);
    int32_t hflag[2] = {0, 0};
    HIPCHK(p, hipMemcpyAsync(hflag, p->flag, sizeof hflag, hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    if (hflag[0]) return fail(p, S3_ERR_INDEX_RANGE, "an entry index lies outside its mode or matrix");
    if (hflag[1]) return fail(p, S3_ERR_INDEX_RANGE, "the item order holds an id outside [0, n_items)");
    // counts |Omega_X^{n,i}| and |Omega_Y^{2,k}|
    for (int n = 0; n < N; ++n) {
        HIPCHK(p, hipMemsetAsync(p->cnt[n], 0, sizeof(int32_t) * p->d.dims[n], st));
        row_counts(buf->x_idx + (int64_t)n * p->nX, p->nX, p->d.dims[n], p->cnt[n], st);
    }
    for (int m = 0; m < M; ++m) {
        HIPCHK(p, hipMemsetAsync(p->cntV[m], 0, sizeof(int32_t) * p->d.mat_cols[m], st));
        row_counts(buf->y_col[m], y_nnz[m], p->d.mat_cols[m], p->cntV[m], st);
    }
    p->det_ready = false;
    p->adj_ready = false;
    if (with_order) {
        // temporaries sit at the end of the carved layout
        char *tmp = (char *)ws + (need - 256 - temp_bytes);  // the offset layout() measured from
        s3_status s = build_det<T>(p, tmp, st);
        if (s != S3_OK) return s;
        p->det_ready = p->adj_ready = true;
    }
    s3_status s = lockfree_build<T>(p->lf, p->d, buf, p->cnt, p->cntV, p->nX, y_nnz, st, p->err);
    if (s != S3_OK) return s;
    HIPCHK(p, hipStreamSynchronize(st));
    HIPCHK(p, hipGetLastError());
    p->bound = true;
    return S3_OK;
}

template <typename T> s3_status loss_impl(s3_plan *p, double *out, hipStream_t st) {
    const int N = p->N, M = p->M;
    double *r = p->red;
    pad_core<T>(p, st);
    std::vector<double> h(kReduceBlocks);
    double sse_t = 0, gg = 0, uu = 0, sse_m = 0, vv = 0;
    {
        const int64_t nb = sq_blocks(p->nX);
        p->ks.sq_err(p, p->b.x_idx, p->b.x_val, p->nX, r, st);
        p->h_red.resize((size_t)nb);
        HIPCHK(p, hipMemcpyAsync(p->h_red.data(), r, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        for (int64_t i = 0; i < nb; ++i) sse_t += p->h_red[(size_t)i];
    }
    hipLaunchKernelGGL(k_sq_rows<T>, dim3(kReduceBlocks), dim3(256), 0, st, (const T *)p->b.G, (int64_t)1,
                       (int)p->K, (const int32_t *)nullptr, r);
    HIPCHK(p, hipMemcpyAsync(h.data(), r, sizeof(double) * kReduceBlocks, hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    for (double v : h) gg += v;
    for (int n = 0; n < N; ++n) {
        hipLaunchKernelGGL(k_sq_rows<T>, dim3(kReduceBlocks), dim3(256), 0, st, (const T *)p->b.U[n],
                           p->d.dims[n], p->d.rank[n], (const int32_t *)p->cnt[n], r);
        HIPCHK(p, hipMemcpyAsync(h.data(), r, sizeof(double) * kReduceBlocks, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        for (double v : h) uu += v;
    }
    for (int m = 0; m < M; ++m) {
        const int c = p->d.mat_mode[m];
        if (p->y_nnz[m] > 0) {
            hipLaunchKernelGGL(k_sq_err_matrix<T>, dim3(kReduceBlocks), dim3(256), 0, st, p->b.y_row[m],
                               p->b.y_col[m], (const T *)p->b.y_val[m], p->y_nnz[m], (const T *)p->b.U[c],
                               (const T *)p->b.V[m], p->d.rank[c], r);
            HIPCHK(p, hipMemcpyAsync(h.data(), r, sizeof(double) * kReduceBlocks, hipMemcpyDeviceToHost, st));
            HIPCHK(p, hipStreamSynchronize(st));
            for (double v : h) sse_m += v;
        }
        hipLaunchKernelGGL(k_sq_rows<T>, dim3(kReduceBlocks), dim3(256), 0, st, (const T *)p->b.V[m],
                           p->d.mat_cols[m], p->d.rank[c], (const int32_t *)p->cntV[m], r);
        HIPCHK(p, hipMemcpyAsync(h.data(), r, sizeof(double) * kReduceBlocks, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        for (double v : h) vv += v;
    }
    HIPCHK(p, hipGetLastError());
    const double ft = sse_t + p->d.lambda_reg * (gg + uu);
    const double fm = sse_m + p->d.lambda_reg * vv;
    out[0] = 0.5 * ft + 0.5 * p->d.lambda_m * fm;
    out[1] = ft;
    out[2] = fm;
    if (!std::isfinite(out[0])) return fail(p, S3_ERR_NONFINITE, "objective is not finite");
    return S3_OK;
}

// synchronous range check of caller-supplied SoA indices (not on the hot path)
// flag: a device int32 (default: the plan's), cleared by a fill kernel
s3_status check_indices(s3_plan *p, const int32_t *idx, int64_t nnz, int modes, const int64_t *lim,
                        hipStream_t st, int32_t *flag = nullptr) {
    if (!flag) flag = p->flag + 2;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, flag, (int64_t)1, (int32_t)0);
    for (int n = 0; n < modes; ++n)
        hipLaunchKernelGGL(k_check_range, dim3(grid_for(nnz, 256, 4096)), dim3(256), 0, st, idx + (int64_t)n * nnz,
                           nnz, lim[n], flag);
    int32_t h = 0;
    HIPCHK(p, hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    if (h) return fail(p, S3_ERR_INDEX_RANGE, "an index lies outside its mode");
    return S3_OK;
}

template <typename T> s3_status rmse_impl(s3_plan *p, double *out, hipStream_t st) {
    if (p->nT == 0) { *out = 0.0; return S3_OK; }
    pad_core<T>(p, st);
    p->ks.sq_err(p, p->b.t_idx, p->b.t_val, p->nT, p->red, st);
    const int64_t nb = sq_blocks(p->nT);
    std::vector<double> h((size_t)nb);
    HIPCHK(p, hipMemcpyAsync(h.data(), p->red, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    HIPCHK(p, hipGetLastError());
    double s = 0;
    for (double v : h) s += v;
    *out = std::sqrt(s / (double)p->nT);
    if (!std::isfinite(*out)) return fail(p, S3_ERR_NONFINITE, "held-out RMSE is not finite");
    return S3_OK;
}

}  // namespace

extern "C" {

s3_status s3_bind(s3_plan *p, const s3_buffers *buf, void *d_ws, size_t ws_bytes, void *stream) {
    if (!p || !buf) return S3_ERR_INVALID_ARG;
    if (!buf->x_idx || !buf->x_val || buf->x_nnz < 1 || buf->t_nnz < 0 || (buf->t_nnz > 0 && (!buf->t_idx || !buf->t_val)))
        return fail(p, S3_ERR_INVALID_ARG, "training entries missing or sizes negative");
    for (int n = 0; n < p->N; ++n)
        if (!buf->U[n]) return fail(p, S3_ERR_INVALID_ARG, "factor U[%d] is null", n);
    if (!buf->G) return fail(p, S3_ERR_INVALID_ARG, "core is null");
    for (int m = 0; m < p->M; ++m) {
        if (!buf->V[m] || buf->y_nnz[m] < 0 || (buf->y_nnz[m] > 0 && (!buf->y_row[m] || !buf->y_col[m] || !buf->y_val[m])))
            return fail(p, S3_ERR_INVALID_ARG, "coupled matrix %d incomplete", m);
    }
    int64_t n_items = buf->x_nnz;
    for (int m = 0; m < p->M; ++m) n_items += buf->y_nnz[m];
    if (n_items > INT32_MAX) return fail(p, S3_ERR_UNSUPPORTED, "more than 2^31 - 1 items");
    p->bound = false;
    hipStream_t st = (hipStream_t)stream;
    return (p->tsize == 8) ? bind_impl<double>(p, buf, d_ws, ws_bytes, st) : bind_impl<float>(p, buf, d_ws, ws_bytes, st);
}

s3_status s3_det_batches(s3_plan *p, int64_t first, int64_t count, double eta, void *stream) {
    if (!p) return S3_ERR_INVALID_ARG;
    if (!p->bound || !p->det_ready) return fail(p, S3_ERR_STATE, "det mode needs s3_bind with an item order");
    if (first < 0 || count < 0 || first + count > p->n_batches)
        return fail(p, S3_ERR_INVALID_ARG, "batch range [%lld, %lld) outside [0, %lld)", (long long)first,
                    (long long)(first + count), (long long)p->n_batches);
    hipStream_t st = (hipStream_t)stream;
    // the caller may have written G since the last call: pad it once, and
    // every batch's core step keeps the padded copy current
    if (count > 0) p->tsize == 8 ? pad_core<double>(p, st) : pad_core<float>(p, st);
    for (int64_t b = first; b < first + count; ++b) {
        if (p->tsize == 8) det_batch<double>(p, b, eta, nullptr, nullptr, nullptr, nullptr, nullptr, st);
        else det_batch<float>(p, b, eta, nullptr, nullptr, nullptr, nullptr, nullptr, st);
    }
    HIPCHK(p, hipGetLastError());
    return S3_OK;
}

s3_status s3_epoch(s3_plan *p, int32_t epoch, int32_t mode, void *stream) {
    if (!p || epoch < 0) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_epoch before s3_bind");
    hipStream_t st = (hipStream_t)stream;
    const double eta = eta_of(p->d, epoch);
    if (!p->ev0) {
        HIPCHK(p, hipEventCreate(&p->ev0));
        HIPCHK(p, hipEventCreate(&p->ev1));
    }
    if (mode == S3_DET_MINIBATCH) {
        if (!p->det_ready) return fail(p, S3_ERR_STATE, "det mode needs s3_bind with an item order");
        p->pev_used = 0;
        HIPCHK(p, hipEventRecord(p->ev0, st));
        s3_status s = s3_det_batches(p, 0, p->n_batches, eta, stream);
        HIPCHK(p, hipEventRecord(p->ev1, st));
        p->last_launches = p->n_batches;
        return s;
    }
    if (mode == S3_LOCKFREE) {
        if (p->lf.H == 0) return fail(p, S3_ERR_UNSUPPORTED, "lock-free mode: rank too large for the LDS tables");
        HIPCHK(p, hipEventRecord(p->ev0, st));
        s3_status s;
        p->pev_used = 0;
        auto round = [&](int64_t f, int64_t c, double e, hipStream_t s_) -> int64_t {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (p->prof && c > 0) {
                e0 = prof_event(p, p->pev_used);
                e1 = prof_event(p, p->pev_used + 1);
                if (e0 && e1) p->pev_used += 2;
                else e0 = e1 = nullptr;
            }
            return p->ks.lf_tensor(p, f, c, e, s_, e0, e1);
        };
        if (p->tsize == 8) {
            pad_core<double>(p, st);
            s = lockfree_epoch<double>(p->lf, p->d, epoch, eta, (double *)p->Gp, st, p->err, round);
        } else {
            pad_core<float>(p, st);
            // matrix-core plans: the core's operand image is formatted once
            // here; each round's apply then rewrites the values it changes
            const bool mx = p->d.contraction == S3_CONTRACT_MATRIX;
            p->lf.apply.mx_img = mx ? p->mx_g : nullptr;
            p->lf.apply.mx_kind = mx ? 1 + (p->N == 4 ? 0 : 2) + (p->d.dtype == S3_BF16 ? 0 : 1) : 0;
            p->ks.mx_format(p, st);
            s = lockfree_epoch<float>(p->lf, p->d, epoch, eta, (float *)p->Gp, st, p->err, round);
        }
        HIPCHK(p, hipEventRecord(p->ev1, st));
        HIPCHK(p, hipGetLastError());
        p->last_launches = p->lf.n_rounds;
        return s;
    }
    return fail(p, S3_ERR_INVALID_ARG, "unknown mode %d", mode);
}

s3_status s3_loss(s3_plan *p, double *out, void *stream) {
    if (!p || !out) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_loss before s3_bind");
    hipStream_t st = (hipStream_t)stream;
    return (p->tsize == 8) ? loss_impl<double>(p, out, st) : loss_impl<float>(p, out, st);
}

s3_status s3_rmse(s3_plan *p, double *out, void *stream) {
    if (!p || !out) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_rmse before s3_bind");
    hipStream_t st = (hipStream_t)stream;
    return (p->tsize == 8) ? rmse_impl<double>(p, out, st) : rmse_impl<float>(p, out, st);
}

s3_status s3_predict(s3_plan *p, const int32_t *idx, int64_t nnz, void *xhat, void *stream) {
    if (!p || (nnz > 0 && (!idx || !xhat)) || nnz < 0) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_predict before s3_bind");
    if (nnz == 0) return S3_OK;
    hipStream_t st = (hipStream_t)stream;
    {
        s3_status v = check_indices(p, idx, nnz, p->N, p->d.dims, st);
        if (v != S3_OK) return v;
    }
    if (p->tsize == 8) pad_core<double>(p, st); else pad_core<float>(p, st);
    p->ks.predict(p, idx, nnz, xhat, p->Gp, st);
    HIPCHK(p, hipGetLastError());
    return S3_OK;
}

s3_status s3_predict_noalloc(s3_plan *p, const int32_t *idx, int64_t nnz, void *xhat, void *stream) {
    if (!p || (nnz > 0 && (!idx || !xhat)) || nnz < 0) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_predict_noalloc before s3_bind");
    const size_t need = 256 + (size_t)p->KP * p->tsize;
    if (need > kStaticScratchBytes)
        return fail(p, S3_ERR_WORKSPACE, "the padded core needs %zu bytes of the %zu-byte static scratch", need,
                    kStaticScratchBytes);
    if (nnz == 0) return S3_OK;
    void *sp = nullptr;
    s3_status s = scratch_ptr(p, &sp);
    if (s != S3_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    s = check_indices(p, idx, nnz, p->N, p->d.dims, st, (int32_t *)sp);
    if (s != S3_OK) return s;
    void *gp = (char *)sp + 256;
    if (p->tsize == 8) pad_core<double>(p, st, gp); else pad_core<float>(p, st, gp);
    p->ks.predict(p, idx, nnz, xhat, gp, st);
    HIPCHK(p, hipGetLastError());
    return S3_OK;
}

s3_status s3_predict_matrix(s3_plan *p, int32_t m, const int32_t *row, const int32_t *col, int64_t nnz,
                            void *yhat, void *stream) {
    if (!p || m < 0 || m >= p->M || nnz < 0 || (nnz > 0 && (!row || !col || !yhat))) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_predict_matrix before s3_bind");
    if (nnz == 0) return S3_OK;
    hipStream_t st = (hipStream_t)stream;
    const int c = p->d.mat_mode[m];
    {
        const int64_t lim_r[1] = {p->d.dims[c]}, lim_c[1] = {p->d.mat_cols[m]};
        s3_status v = check_indices(p, row, nnz, 1, lim_r, st);
        if (v == S3_OK) v = check_indices(p, col, nnz, 1, lim_c, st);
        if (v != S3_OK) return v;
    }
    if (p->tsize == 8)
        hipLaunchKernelGGL(k_predict_matrix<double>, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, st, row, col, nnz,
                           (const double *)p->b.U[c], (const double *)p->b.V[m], p->d.rank[c], (double *)yhat);
    else
        hipLaunchKernelGGL(k_predict_matrix<float>, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, st, row, col, nnz,
                           (const float *)p->b.U[c], (const float *)p->b.V[m], p->d.rank[c], (float *)yhat);
    HIPCHK(p, hipGetLastError());
    return S3_OK;
}

s3_status s3_backward(s3_plan *p, const void *gx, const void *const *gy, void *const *dU, void *dG,
                      void *const *dV, void *stream) {
    if (!p || !dU || !dG || (p->M > 0 && !dV)) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_backward before s3_bind");
    for (int n = 0; n < p->N; ++n)
        if (!dU[n]) return S3_ERR_INVALID_ARG;
    for (int m = 0; m < p->M; ++m)
        if (!dV[m]) return S3_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = p->tsize == 8;
    if (!p->adj_ready) {
        s3_status s = f64 ? build_adjoint_order<double>(p, st) : build_adjoint_order<float>(p, st);
        if (s != S3_OK) return s;
    }
    for (int n = 0; n < p->N; ++n)
        f64 ? fill<double>(dU[n], p->d.dims[n] * p->d.rank[n], 0.0, st) : fill<float>(dU[n], p->d.dims[n] * p->d.rank[n], 0.0, st);
    f64 ? fill<double>(dG, p->K, 0.0, st) : fill<float>(dG, p->K, 0.0, st);
    for (int m = 0; m < p->M; ++m) {
        const int64_t cnt = p->d.mat_cols[m] * p->d.rank[p->d.mat_mode[m]];
        f64 ? fill<double>(dV[m], cnt, 0.0, st) : fill<float>(dV[m], cnt, 0.0, st);
    }
    const void *const nogy[S3_MAX_MATRICES] = {nullptr, nullptr, nullptr, nullptr};
    const void *const *gyv = gy ? gy : nogy;
    f64 ? pad_core<double>(p, st) : pad_core<float>(p, st);
    for (int64_t b = 0; b < p->n_batches; ++b) {
        if (f64) det_batch<double>(p, b, 0.0, gx, gyv, dU, dG, dV, st);
        else det_batch<float>(p, b, 0.0, gx, gyv, dU, dG, dV, st);
    }
    HIPCHK(p, hipGetLastError());
    return S3_OK;
}

}  // extern "C"

namespace {
// the bound parameter buffer (which = 0: U[index], 1: G, 2: V[index]) and
// its element count, or an error when no such parameter exists
s3_status param_slot(s3_plan *p, int32_t which, int32_t index, void **ptr, int64_t *count) {
    if (which == 0 && index >= 0 && index < p->N) {
        *ptr = p->b.U[index];
        *count = p->d.dims[index] * p->d.rank[index];
    } else if (which == 1) {
        *ptr = p->b.G;
        *count = p->K;
    } else if (which == 2 && index >= 0 && index < p->M) {
        *ptr = p->b.V[index];
        *count = p->d.mat_cols[index] * p->d.rank[p->d.mat_mode[index]];
    } else {
        return fail(p, S3_ERR_INVALID_ARG, "unknown parameter (%d, %d)", which, index);
    }
    return S3_OK;
}
}  // namespace

extern "C" {

s3_status s3_export(s3_plan *p, int32_t which, int32_t index, double *host_dst, size_t bytes, void *stream) {
    if (!p || !host_dst) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_export before s3_bind");
    void *src = nullptr;
    int64_t count = 0;
    s3_status s = param_slot(p, which, index, &src, &count);
    if (s != S3_OK) return s;
    if (bytes != (size_t)count * sizeof(double))
        return fail(p, S3_ERR_INVALID_ARG, "export needs %lld bytes", (long long)(count * 8));
    hipStream_t st = (hipStream_t)stream;
    if (p->tsize == 8) {
        HIPCHK(p, hipMemcpyAsync(host_dst, src, bytes, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
    } else {
        std::vector<float> tmp((size_t)count);
        HIPCHK(p, hipMemcpyAsync(tmp.data(), src, sizeof(float) * count, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        for (int64_t i = 0; i < count; ++i) host_dst[i] = (double)tmp[(size_t)i];
    }
    return S3_OK;
}

s3_status s3_import(s3_plan *p, int32_t which, int32_t index, const double *host_src, size_t bytes,
                    void *stream) {
    if (!p || !host_src) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_import before s3_bind");
    void *dst = nullptr;
    int64_t count = 0;
    s3_status s = param_slot(p, which, index, &dst, &count);
    if (s != S3_OK) return s;
    if (bytes != (size_t)count * sizeof(double))
        return fail(p, S3_ERR_INVALID_ARG, "import needs %lld bytes", (long long)(count * 8));
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(host_src[i]))
            return fail(p, S3_ERR_NONFINITE, "import: value %lld is not finite", (long long)i);
    hipStream_t st = (hipStream_t)stream;
    if (p->tsize == 8) {
        HIPCHK(p, hipMemcpyAsync(dst, host_src, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(p, hipStreamSynchronize(st));
    } else {
        // round to nearest FP32 (the masters of FP32 and BF16-operand plans)
        std::vector<float> tmp((size_t)count);
        for (int64_t i = 0; i < count; ++i) tmp[(size_t)i] = (float)host_src[i];
        HIPCHK(p, hipMemcpyAsync(dst, tmp.data(), sizeof(float) * count, hipMemcpyHostToDevice, st));
        HIPCHK(p, hipStreamSynchronize(st));
    }
    return S3_OK;
}

}  // extern "C"

namespace {
template <typename T> s3_status orthogonalize_impl(s3_plan *p, hipStream_t st) {
    const int N = p->N;
    const int *J = p->d.rank;
    HIPCHK(p, hipMemsetAsync(p->flag, 0, sizeof(int32_t), st));
    for (int n = 0; n < N; ++n) {
        double *R = p->qr_R + (size_t)n * 3 * kQrJ * kQrJ, *Rinv = R + kQrJ * kQrJ, *Rtot = Rinv + kQrJ * kQrJ;
        const int64_t I = p->d.dims[n];
        const int nb = (int)std::min<int64_t>(kQrBlocks, std::max<int64_t>(1, (I + kQrRows - 1) / kQrRows));
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_gram<T>, dim3(nb), dim3(256), 0, st, (const T *)p->b.U[n], I, J[n], p->qr_part);
            hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, st, (const double *)p->qr_part, nb, J[n], R, Rinv,
                               Rtot, pass == 0 ? 1 : 0, p->flag);
            hipLaunchKernelGGL(k_apply_rinv<T>, dim3(grid_for(I, 256, 4096)), dim3(256), 0, st, (T *)p->b.U[n], I,
                               J[n], (const double *)Rinv);
        }
        // G <- G x_n R
        HIPCHK(p, hipMemcpyAsync(p->qr_G, p->b.G, sizeof(T) * p->K, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_core_mode_mul<T>, dim3(grid_for(p->K, 256, 64)), dim3(256), 0, st, (const T *)p->qr_G,
                           (T *)p->b.G, N, J[0], J[1], J[2], N > 3 ? J[3] : 1, n, (const double *)Rtot);
    }
    for (int m = 0; m < p->M; ++m) {
        const int c = p->d.mat_mode[m];
        const double *Rtot = p->qr_R + (size_t)c * 3 * kQrJ * kQrJ + 2 * kQrJ * kQrJ;
        hipLaunchKernelGGL(k_rows_times_rt<T>, dim3(grid_for(p->d.mat_cols[m], 256, 4096)), dim3(256), 0, st,
                           (T *)p->b.V[m], (int64_t)p->d.mat_cols[m], J[c], Rtot);
    }
    HIPCHK(p, hipGetLastError());
    int32_t bad = 0;
    HIPCHK(p, hipMemcpyAsync(&bad, p->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    if (bad) return fail(p, S3_ERR_NONFINITE, "orthogonalisation: a factor matrix is not numerically full rank");
    return S3_OK;
}
// SplitMix64's output function on the host (same definition as the device
// one in kernels.hpp), to derive each parameter's counter key
uint64_t host_splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

extern "C" {

s3_status s3_orthogonalize(s3_plan *p, void *stream) {
    if (!p) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_orthogonalize before s3_bind");
    if (p->d.core_kind == S3_CORE_CP)
        return fail(p, S3_ERR_UNSUPPORTED, "orthogonalisation makes a hyper-diagonal core dense");
    for (int n = 0; n < p->N; ++n)
        if (p->d.rank[n] > kQrJ || p->d.rank[n] > p->d.dims[n])
            return fail(p, S3_ERR_UNSUPPORTED, "orthogonalisation needs J_n <= min(16, I_n)");
    hipStream_t st = (hipStream_t)stream;
    return p->tsize == 8 ? orthogonalize_impl<double>(p, st) : orthogonalize_impl<float>(p, st);
}

s3_status s3_init_params(s3_plan *p, uint64_t seed, double sigma, void *stream) {
    if (!p || !(sigma >= 0.0) || !std::isfinite(sigma)) return S3_ERR_INVALID_ARG;
    if (!p->bound) return fail(p, S3_ERR_STATE, "s3_init_params before s3_bind");
    hipStream_t st = (hipStream_t)stream;
    // parameter q: U^(n) is q = n, G is q = N, V_m is q = N + 1 + m; its
    // counters start at the SplitMix64 mix of seed + (q + 1) * golden gamma
    auto one = [&](void *ptr, int64_t count, int q) {
        if (count <= 0) return;
        const uint64_t key = host_splitmix64_mix(seed + 0x9E3779B97F4A7C15ull * (uint64_t)(q + 1));
        const int64_t pairs = (count + 1) / 2;
        if (p->tsize == 8)
            hipLaunchKernelGGL(k_init_normal<double>, dim3(grid_for(pairs, 256, 4096)), dim3(256), 0, st,
                               (double *)ptr, count, key, sigma);
        else
            hipLaunchKernelGGL(k_init_normal<float>, dim3(grid_for(pairs, 256, 4096)), dim3(256), 0, st,
                               (float *)ptr, count, key, sigma);
    };
    for (int n = 0; n < p->N; ++n) one(p->b.U[n], p->d.dims[n] * p->d.rank[n], n);
    one(p->b.G, p->K, p->N);
    for (int m = 0; m < p->M; ++m) one(p->b.V[m], p->d.mat_cols[m] * p->d.rank[p->d.mat_mode[m]], p->N + 1 + m);
    HIPCHK(p, hipGetLastError());
    return S3_OK;
}

s3_status s3_set_profiling(s3_plan *p, int32_t on) {
    if (!p) return S3_ERR_INVALID_ARG;
    p->prof = on != 0;
    return S3_OK;
}

s3_status s3_last_epoch_profile(const s3_plan *cp, double *kernel_ms, int64_t *launches) {
    s3_plan *p = const_cast<s3_plan *>(cp);
    if (!p || !kernel_ms || !launches) return S3_ERR_INVALID_ARG;
    if (!p->ev0) return fail(p, S3_ERR_STATE, "no epoch has run");
    HIPCHK(p, hipEventSynchronize(p->ev1));
    if (p->prof && p->pev_used >= 2) {
        double total = 0.0;
        for (size_t k = 0; k + 1 < p->pev_used; k += 2) {
            float ms = 0.f;
            HIPCHK(p, hipEventElapsedTime(&ms, p->pev[k], p->pev[k + 1]));
            total += ms;
        }
        *kernel_ms = total;
        *launches = (int64_t)(p->pev_used / 2);
        return S3_OK;
    }
    float ms = 0.f;
    HIPCHK(p, hipEventElapsedTime(&ms, p->ev0, p->ev1));
    *kernel_ms = ms;
    *launches = p->last_launches;
    return S3_OK;
}

}  // extern "C"
