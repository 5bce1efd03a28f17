// Internal to the library: the plan object behind the C ABI and the
// per-shape kernel sets its entry points dispatch to.  Every translation unit
// of the library includes it; the kernel sets are compiled in separate units
// (sets_*.hip) so that they build in parallel.
#pragma once
#include "s3cmtf.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lockfree.hpp"
#include "qr.hpp"

namespace s3 {

constexpr int kReduceBlocks = 1024;  // fixed grid => fixed reduction order

struct Group {
    uint64_t *contrib = nullptr;  // sorted (goff | coff << 32)
    int64_t *seg_start = nullptr; // [nseg + 1]
    int32_t *seg_row = nullptr;   // [nseg]
    int32_t *med_ids = nullptr;   // segments of (kShortSeg, kLongSeg] contributions
    int32_t *long_ids = nullptr;  // longer segments, in order
    int32_t *long_fp = nullptr;   // first piece of each long segment (+ end)
    int64_t *pc0 = nullptr, *pc1 = nullptr;  // pieces of the long segments
    int64_t n_valid = 0;
    int64_t nseg = 0;
    std::vector<int64_t> h_boff;  // per-batch ranges: segments, medium, long, pieces
    std::vector<int64_t> h_moff, h_loff, h_poff;
    int J = 0;
    int64_t rows = 0;
};

// bump allocator over the workspace; with base == nullptr it only measures
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <typename X> X *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        X *p = base ? (X *)(base + off) : nullptr;
        off += count * sizeof(X);
        return p;
    }
};

}  // namespace s3


// the library's own namespace is used unqualified in its internal units
using namespace s3;

// ------------------------------------------------------------------ dispatch

struct KernelSet {
    void (*det_entries)(s3_plan *, const int32_t *, int64_t, int64_t, const void *, const void *, int64_t,
                        hipStream_t, hipEvent_t, hipEvent_t);
    void (*core_partial)(s3_plan *, const int32_t *, int64_t, hipStream_t);
    void (*sq_err)(s3_plan *, const int32_t *, const void *, int64_t, double *, hipStream_t);
    void (*predict)(s3_plan *, const int32_t *, int64_t, void *, const void *, hipStream_t);  // Gp: padded core
    // returns the number of tensor workgroups (partial tables) it launched
    int64_t (*lf_tensor)(s3_plan *, int64_t, int64_t, double, hipStream_t, hipEvent_t, hipEvent_t);
    void (*mx_format)(s3_plan *, hipStream_t);  // matrix-core sets: core operands from Gp into mx_g
    int det_chunk;  // tensor entries per det block and core chunk
};

struct s3_plan {
    s3_desc d{};
    int N = 0, M = 0, JP = 0;
    bool exact = false;  // every rank equals JP
    int64_t K = 1, KP = 1;
    size_t tsize = 4;  // sizeof compute type
    bool bound = false;
    s3_buffers b{};
    KernelSet ks{};
    std::string err;
    // workspace arrays
    int32_t *cnt[S3_MAX_ORDER] = {};
    int32_t *cntV[S3_MAX_MATRICES] = {};
    void *Gp = nullptr;
    void *mx_g = nullptr;  // the padded core in the matrix-core operand layout
    int32_t *flag = nullptr;
    double *red = nullptr;  // reduction partials
    int64_t n_red = 0;
    std::vector<double> h_red;
    // det structures
    int64_t nX = 0, nT = 0, n_items = 0, n_batches = 0;
    int64_t y_nnz[S3_MAX_MATRICES] = {};
    int64_t mat_begin[S3_MAX_MATRICES] = {};
    int32_t *sorted_ids = nullptr;
    int32_t *bidx = nullptr;  // items' indices in det item order [N][n_items]
    void *bval = nullptr;     // items' values in det item order [n_items]
    std::vector<int64_t> h_type_off;
    Group grp[S3_MAX_ORDER + S3_MAX_MATRICES];
    void *scr = nullptr;
    int64_t t_stride = 0, RJ = 0;
    int64_t m_base[S3_MAX_MATRICES] = {}, m_stride[S3_MAX_MATRICES] = {};
    void *part = nullptr, *part_curv = nullptr;
    int64_t max_chunks = 0;
    void *rows_part = nullptr;  // piece sums of the long segments of one batch
    bool det_ready = false;   // det structures built from the caller's item order
    bool adj_ready = false;   // det structures built (from that order, or from the storage order)
    void *ws_base = nullptr;  // the bound workspace
    size_t ws_bytes = 0;
    size_t det_carve_off = 0;  // where the det structures start in it
    // lock-free structures
    LockFreeState lf;
    // orthogonalisation: Gram partials, per mode R / R^-1 / running R, a core copy
    double *qr_part = nullptr, *qr_R = nullptr;
    void *qr_G = nullptr;
    // profiling
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
    int64_t last_launches = 0;
    bool prof = false;
    std::vector<hipEvent_t> pev;  // pairs around the dominant kernel
    size_t pev_used = 0;
};

namespace s3 {

// blocks of the one-entry-per-thread squared-error kernel
inline int64_t sq_blocks(int64_t nnz) { return std::max<int64_t>(1, (nnz + 255) / 256); }

inline int grid_for(int64_t n, int tpb, int64_t cap = 65535 * 4) {
    int64_t g = (n + tpb - 1) / tpb;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <typename T> inline TensorArgs<T> tensor_args(const s3_plan *p, const int32_t *idx, const void *val,
                                                int64_t nnz) {
    TensorArgs<T> a{};
    a.idx = idx;
    a.nnz = nnz;
    a.val = (const T *)val;
    for (int n = 0; n < p->N; ++n) {
        a.U[n] = (T *)p->b.U[n];
        a.J[n] = p->d.rank[n];
        a.cnt[n] = p->cnt[n];
    }
    a.lambda_reg = (T)p->d.lambda_reg;
    return a;
}

// CT: the per-entry contraction (reuse, naive ablation, or the
// hyper-diagonal CP core)
template <int N, int JP, typename T, int CT = kReuse> struct Impl {
    // the batch's tensor entries (t_blocks chunks, 0 when the adjoint has
    // no tensor sensitivity) and coupled-matrix entries (*mats) in one launch;
    // e0/e1 (profiling, may be null) take the dispatch's own start and end
    static void det_entries(s3_plan *p, const int32_t *ids, int64_t nt, int64_t t_blocks, const void *gx,
                            const void *mats, int64_t blocks, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
        auto a = tensor_args<T>(p, p->b.x_idx, p->b.x_val, p->nX);
        const DetMatArgs<T> &B = *(const DetMatArgs<T> *)mats;
        const int64_t t0 = ids - p->sorted_ids;  // the batch's first tensor item position
        const int32_t *bidx = p->bidx + t0;
        const T *bval = (const T *)p->bval + t0;
        if (gx)
            hipExtLaunchKernelGGL((k_det_entries<N, JP, T, true, CT>), dim3((unsigned)blocks), dim3(kChunk), 0, st,
                                  e0, e1, 0, a, ids, nt, t_blocks, (const T *)p->Gp, (T *)p->scr, p->t_stride,
                                  (const T *)gx, (T *)p->part, (T *)p->part_curv, B, bidx, bval, p->n_items,
                                  (const void *)p->mx_g);
        else
            hipExtLaunchKernelGGL((k_det_entries<N, JP, T, false, CT>), dim3((unsigned)blocks), dim3(kChunk), 0, st,
                                  e0, e1, 0, a, ids, nt, t_blocks, (const T *)p->Gp, (T *)p->scr, p->t_stride,
                                  (const T *)nullptr, (T *)p->part, (T *)p->part_curv, B, bidx, bval, p->n_items,
                                  (const void *)p->mx_g);
    }
    // FP64 Tucker core partials (the other cores are formed in det_entries)
    static void core_partial(s3_plan *p, const int32_t *ids, int64_t nt, hipStream_t st) {
        if constexpr (!det_fused_core<T, CT>()) {
            constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
            constexpr int TPB = ((TAIL + 63) / 64) * 64;
            auto a = tensor_args<T>(p, p->b.x_idx, p->b.x_val, p->nX);
            const int64_t nch = (nt + kChunk - 1) / kChunk;
            hipLaunchKernelGGL((k_core_partial<N, JP, T>), dim3((unsigned)nch), dim3(TPB), 0, st, a, ids, nt,
                               (const T *)p->scr, p->t_stride, (T *)p->part, (T *)p->part_curv);
        }
    }
    static void sq_err(s3_plan *p, const int32_t *idx, const void *val, int64_t nnz, double *part,
                       hipStream_t st) {
        auto a = tensor_args<T>(p, idx, val, nnz);
        hipLaunchKernelGGL((k_sq_err_tensor<N, JP, T, CT>), dim3(sq_blocks(nnz)), dim3(256), 0, st, a,
                           (const T *)p->Gp, part);
    }
    static void predict(s3_plan *p, const int32_t *idx, int64_t nnz, void *out, const void *Gp, hipStream_t st) {
        auto a = tensor_args<T>(p, idx, nullptr, nnz);
        hipLaunchKernelGGL((k_predict<N, JP, T, CT>), dim3(grid_for(nnz, 256, 1ll << 30)), dim3(256), 0, st, a,
                           (const T *)Gp, (T *)out);
    }
    static int64_t lf_tensor(s3_plan *p, int64_t first, int64_t count, double eta, hipStream_t st, hipEvent_t e0,
                             hipEvent_t e1) {
        if (p->exact)
            return lockfree_tensor_launch<N, JP, T, true, CT>(p->lf, tensor_args<T>(p, p->b.x_idx, p->b.x_val, p->nX),
                                                          (const T *)p->Gp, first, count, (T)eta, st, e0, e1,
                                                          p->mx_g);
        else
            return lockfree_tensor_launch<N, JP, T, false, CT>(p->lf, tensor_args<T>(p, p->b.x_idx, p->b.x_val, p->nX),
                                                           (const T *)p->Gp, first, count, (T)eta, st, e0, e1,
                                                           p->mx_g);
    }
    static void mx_format(s3_plan *p, hipStream_t st) {
        if constexpr (is_mx(CT) && mfma_shape<N, JP>() && std::is_same<T, float>::value) {
            constexpr int OP = (CT == kMfma16) ? kOpBF16 : kOpF32;
            constexpr int n = mfma_core_count<N, JP, OP>();
            hipLaunchKernelGGL((k_mx_format<N, JP, OP>), dim3((n + 255) / 256), dim3(256), 0, st, (const float *)p->Gp,
                               p->mx_g);
        }
    }
};

template <int N, int JP, typename T, int CT = kReuse> KernelSet make_set() {
    using I = Impl<N, JP, T, CT>;
    return KernelSet{&I::det_entries, &I::core_partial, &I::sq_err, &I::predict, &I::lf_tensor, &I::mx_format,
                     det_chunk<T, CT>()};
}

// kernel sets by element type and contraction; false when the shape is not built
bool pick_reuse_f32_3(int JP, KernelSet *ks);
bool pick_reuse_f32_4(int JP, KernelSet *ks);
bool pick_reuse_f64(int N, int JP, KernelSet *ks);
bool pick_cp(bool f64, int N, int JP, KernelSet *ks);
bool pick_naive(bool f64, int N, int JP, KernelSet *ks);
bool pick_mx(bool bf16, int N, int JP, KernelSet *ks);

}  // namespace s3
