// gfx950 kernels for sparse coupled Tucker SGD.
//
// Hot path of one deterministic mini-batch step (item order cut into
// batches; all gradients at the batch-start values), three launches:
//   k_det_entries     per tensor entry (one lane, or a quarter of the core
//                     on each of four wavefronts): gather the N factor rows,
//                     single pass over the core (contract.hpp) -> x~, e,
//                     w_n; write the row gradients of Eq (8) and the scalar
//                     -e to a per-batch scratch row; then the chunk's core
//                     gradient sum_t (-e_t) u^(1)_t o ... o u^(N)_t over its
//                     64 or 256 entries (FP32 matrix cores, or the hyper-diagonal
//                     core on the VALU; an FP64 Tucker core takes
//                     k_core_partial).  Later blocks: one lane per
//                     coupled-matrix entry (u.v, e, both row gradients)
//   k_rows_reduce     every touched row's contributions summed in a fixed
//                     order and applied (-eta * sum, damped): a lane, a
//                     wavefront or pieces of a workgroup each, by row
//                     length; its last blocks sum the chunk partials in
//                     order, add the regulariser and apply the core step
//   k_rows_finish     the pieces of the longest rows, in order
// All reductions have a fixed order, so a det-mode run is bitwise
// reproducible.
#pragma once
#include <cstdint>

#include "common.hpp"
#include "contract.hpp"
#include "mfma.hpp"
#include "sort.hpp"

namespace s3 {

constexpr int kMaxN = 4;
constexpr int kMaxM = 4;
constexpr int kChunk = 256;  // entries per core-gradient chunk

template <typename T> struct TensorArgs {
    const int32_t *idx;  // [N][nnz]
    int64_t nnz;
    const T *val;
    T *U[kMaxN];
    int J[kMaxN];
    const int32_t *cnt[kMaxN];
    T lambda_reg;
};

// ----------------------------------------------------------------------- prep

static __global__ void k_check_range(const int32_t *__restrict__ idx, int64_t n, int64_t limit,
                              int32_t *__restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < n; i += stride) {
        const int32_t v = idx[i];
        bad |= (v < 0) | ((int64_t)v >= limit);
    }
    if (bad) atomicOr(flag, 1);
}

// key = batch * (M + 1) + type (0 tensor, m + 1 matrix m); value = item id
static __global__ void k_order_keys(const int32_t *__restrict__ order, int64_t n, int64_t batch,
                             int64_t nX, int32_t M, const int64_t *__restrict__ mat_end,
                             uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += stride) {
        const int64_t id = order ? order[t] : t;  // null: the storage order
        int type = 0;
        if (id >= nX) {
            type = 1;
            for (int m = 0; m < M; ++m)
                if (id >= mat_end[m]) type = m + 2;
        }
        key[t] = (uint32_t)((t / batch) * (M + 1) + type);
        val[t] = (int32_t)id;
    }
}

// off[k] = first position whose key >= k, for k in [0, nkeys]; keys sorted
template <typename K>
__global__ void k_bounds(const K *__restrict__ key, int64_t n, int64_t nkeys,
                         int64_t *__restrict__ off) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; p <= n; p += stride) {
        const int64_t lo = (p == 0) ? -1 : (int64_t)key[p - 1];
        const int64_t hi = (p == n) ? nkeys : (int64_t)key[p];
        for (int64_t k = lo + 1; k <= hi && k <= nkeys; ++k) off[k] = p;
    }
}

// Contributions of every sorted item position to one parameter group.
// Group g < N: rows of U^(g) (tensor entries, and entries of matrices
// coupled to mode g).  Group N + m: rows of V_m.  key = (batch << rbits) |
// row, val = gradient offset | (curvature offset << 32) into the batch
// scratch.  Positions that do not touch the group get key nb << rbits, above
// every real key, and sort last.
struct GroupArgs {
    const int32_t *sorted_ids;   // item ids grouped by (batch, type)
    const uint32_t *sorted_keys; // their (batch, type) keys
    const int64_t *type_off;     // first position of each (batch, type) key
    int64_t n;
    int32_t M;
    int32_t N;
    int32_t group;
    int64_t nX;
    const int32_t *x_idx;
    int64_t x_nnz;
    const int32_t *y_row[kMaxM];
    const int32_t *y_col[kMaxM];
    int64_t mat_begin[kMaxM];
    int32_t mat_mode[kMaxM];
    int64_t t_stride;      // floats per tensor scratch row
    int64_t t_goff;        // offset of this group's gradient in a tensor row
    int64_t t_coff;        // offset of this group's curvature in a tensor row
    int64_t m_base[kMaxM]; // start of each matrix's scratch region
    int64_t m_stride[kMaxM];
    int32_t m_J[kMaxM];
    int32_t rbits;         // bits of a row index in the sort key
    int64_t nb;            // batches; key nb << rbits marks "no contribution"
};

static __global__ void k_group_contrib(GroupArgs a, uint64_t *__restrict__ key_out,
                                uint64_t *__restrict__ val_out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; p < a.n; p += stride) {
        const uint32_t k = a.sorted_keys[p];
        const int64_t b = k / (a.M + 1);
        const int type = (int)(k % (a.M + 1));
        const int64_t slot = p - a.type_off[k];
        const int64_t id = a.sorted_ids[p];
        uint64_t kk = (uint64_t)a.nb << a.rbits, vv = 0;
        if (type == 0) {
            if (a.group < a.N) {
                const int64_t row = a.x_idx[(int64_t)a.group * a.x_nnz + id];
                const int64_t go = slot * a.t_stride + a.t_goff;
                const int64_t co = slot * a.t_stride + a.t_coff;
                kk = ((uint64_t)b << a.rbits) | (uint64_t)row;
                vv = (uint64_t)go | ((uint64_t)co << 32);
            }
        } else {
            const int m = type - 1;
            const int64_t e = id - a.mat_begin[m];
            const int64_t base = a.m_base[m] + slot * a.m_stride[m];
            const int J = a.m_J[m];
            if (a.group == a.mat_mode[m]) {
                kk = ((uint64_t)b << a.rbits) | (uint64_t)a.y_row[m][e];
                vv = (uint64_t)base | ((uint64_t)(base + 2 * J) << 32);
            } else if (a.group == a.N + m) {
                kk = ((uint64_t)b << a.rbits) | (uint64_t)a.y_col[m][e];
                vv = (uint64_t)(base + J) | ((uint64_t)(base + 2 * J + 1) << 32);
            }
        }
        key_out[p] = kk;
        val_out[p] = vv;
    }
}

static __global__ void k_seg_flags(const uint64_t *__restrict__ key, int64_t n, int32_t *__restrict__ flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; p < n; p += stride) flag[p] = (p == 0 || key[p] != key[p - 1]) ? 1 : 0;
}

// seg_id = inclusive scan of flags - 1
static __global__ void k_seg_write(const uint64_t *__restrict__ key, const int32_t *__restrict__ flag,
                            const int32_t *__restrict__ seg_id, int64_t n,
                            int64_t *__restrict__ seg_start, int32_t *__restrict__ seg_row,
                            uint32_t *__restrict__ seg_batch, int rbits) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; p < n; p += stride) {
        if (flag[p]) {
            const int64_t s = seg_id[p] - 1;
            seg_start[s] = p;
            seg_row[s] = (int32_t)(key[p] & ((1ull << rbits) - 1ull));
            seg_batch[s] = (uint32_t)(key[p] >> rbits);
        }
        if (p == n - 1) seg_start[seg_id[p]] = n;
    }
}

// --------------------------------------------------------------- core padding

// copy the core J_1 x .. x J_N into a zero-padded JP^N row-major buffer
template <typename T>
__global__ void k_pad_core(const T *__restrict__ G, T *__restrict__ Gp, int N, int JP, int J0,
                           int J1, int J2, int J3) {
    const int Js[4] = {J0, J1, J2, J3};
    int KP = 1;
    for (int n = 0; n < N; ++n) KP *= JP;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < KP; p += gridDim.x * blockDim.x) {
        int rem = p, src = 0, mul = 1;
        bool inside = true;
        int jj[4];
        for (int n = N - 1; n >= 0; --n) { jj[n] = rem % JP; rem /= JP; }
        for (int n = N - 1; n >= 0; --n) {
            inside &= jj[n] < Js[n];
            src += jj[n] * mul;
            mul *= Js[n];
        }
        Gp[p] = inside ? G[src] : T(0);
    }
}

// ------------------------------------------------------------- row loading

// EXACT: every rank equals JP, so rows load without predicates (the
// compiler then merges them into wide vector loads)
template <int N, int JP, typename T, bool EXACT = false>
S3_DEV void load_rows(const TensorArgs<T> &A, int64_t e, T (&u)[N][JP], int32_t (&rows)[N]) {
#pragma unroll
    for (int n = 0; n < N; ++n) {
        rows[n] = A.idx[(int64_t)n * A.nnz + e];
        const T *r = A.U[n] + (int64_t)rows[n] * (EXACT ? JP : A.J[n]);
#pragma unroll
        for (int k = 0; k < JP; ++k) u[n][k] = (EXACT || k < A.J[n]) ? r[k] : T(0);
    }
}

// ----------------------------------------------------- det: batch-ordered items

// Bind time: every item's indices and value copied into the det item order
// (position p holds item sorted_ids[p]), so the batch kernels read them
// contiguously instead of through the id: a tensor item's N mode indices go
// to bidx[n][p] and its value to bval[p]; a matrix item's row and column to
// bidx[0][p] and bidx[1][p] and its value to bval[p].
template <typename T> struct GatherArgs {
    const int32_t *ids;
    int64_t n, nX;
    int N, M;
    const int32_t *x_idx;  // [N][nX]
    const T *x_val;
    int64_t mat_begin[kMaxM];
    const int32_t *y_row[kMaxM], *y_col[kMaxM];
    const T *y_val[kMaxM];
    int32_t *bidx;  // [N][n]
    T *bval;        // [n]
};

template <typename T> __global__ void k_gather_items(GatherArgs<T> a) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = a.ids[p];
        if (id < a.nX) {
            for (int n = 0; n < a.N; ++n) a.bidx[(int64_t)n * a.n + p] = a.x_idx[(int64_t)n * a.nX + id];
            a.bval[p] = a.x_val[id];
        } else {
            int m = 0;
            for (int h = 1; h < a.M; ++h)
                if (id >= a.mat_begin[h]) m = h;
            const int64_t e = id - a.mat_begin[m];
            a.bidx[p] = a.y_row[m][e];
            a.bidx[a.n + p] = a.y_col[m][e];
            a.bval[p] = a.y_val[m][e];
        }
    }
}

// ------------------------------------------------------------ det: entries

// Coupled-matrix entries of one det batch (every matrix in the same launch).
template <typename T> struct DetMatrix {
    const int32_t *ids;       // the batch's sorted item ids of this matrix
    int64_t n, id_base;       // entries in the batch; item id of entry 0
    const int32_t *row, *col; // the batch's rows and columns, in item order
    const T *val, *Uc, *V;    // the batch's values, in item order
    const int32_t *cntV;
    const T *gy;              // adjoint upstream gradient; null: training
    T *scr;                   // scratch rows of this matrix
    int J;
    int64_t b0;               // first block of this matrix in the launch
};

template <typename T> struct DetMatArgs {
    DetMatrix<T> m[kMaxM];
    int M;
    T lambda_m, lambda_reg;
};

// One lane per coupled-matrix entry.  Scratch row: [ g_u (J) | g_v (J) | L_u | L_v ].
// The rows are read with the largest rank unrolled and predicated, so all
// their loads are in flight at once.
template <typename T>
S3_DEV void det_matrix_entry(const DetMatrix<T> &d, int64_t s, T lambda_m, T lambda_reg) {
    constexpr int JM = 16;  // largest rank
    const int J = d.J;
    const int32_t col = d.col[s];
    const T *pu = d.Uc + (int64_t)d.row[s] * J;
    const T *pv = d.V + (int64_t)col * J;
    const T y = d.gy ? d.gy[(int64_t)d.ids[s] - d.id_base] : d.val[s];
    const T cv = d.gy ? T(0) : (T)d.cntV[col];
    T u[JM], v[JM];
#pragma unroll
    for (int k = 0; k < JM; ++k) {
        u[k] = k < J ? pu[k] : T(0);
        v[k] = k < J ? pv[k] : T(0);
    }
    T yh = T(0), uu = T(0), vv = T(0);
#pragma unroll
    for (int k = 0; k < JM; ++k) {
        yh = fmaT(u[k], v[k], yh);
        uu = fmaT(u[k], u[k], uu);
        vv = fmaT(v[k], v[k], vv);
    }
    const bool train = (d.gy == nullptr);
    // training: d/du = -lm e v, d/dv = -lm e u + lm reg v; adjoint: gy v, gy u
    const T q = train ? -lambda_m * (y - yh) : y;
    const T rv = train ? lambda_m * lambda_reg / cv : T(0);
    T *out = d.scr + s * (2 * J + 2);
#pragma unroll
    for (int k = 0; k < JM; ++k) {
        if (k < J) {
            out[k] = q * v[k];
            out[J + k] = fmaT(q, u[k], rv * v[k]);
        }
    }
    out[2 * J] = lambda_m * vv;
    out[2 * J + 1] = fmaT(lambda_m, uu, rv);
}

// Core gradient of one 256-entry tile on the FP32 matrix cores:
//   C[j1][tau] = sum_t (q u^(1))_t[j1] * (u^(2) o ... o u^(N))_t[tau]
// (K = 256 entries, or 64 in the split det form) as a (16 x K) x (K x 16
// n-tiles) product with v_mfma_f32_16x16x4f32
// (A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, D[4 (l / 16) + r][l % 16]
// in lane l, register r).  M = j1 (JP <= 16, zero padded), K = the tile's
// entries, N = tail index tau; wave w takes n-tiles w, w + 4, ...; the
// Khatri-Rao operand is formed from the LDS-staged rows as it is consumed.
typedef float s3_v4f __attribute__((ext_vector_type(4)));

template <int N, int JP, int K = kChunk>
S3_DEV void core_tile_mfma(const float *s_q, const float *s_u, float *core, bool add = false) {
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int NT = (TAIL + 15) / 16;                 // n-tiles
    constexpr int NW = kChunk / kWave;                    // waves of the 256-thread block
    constexpr int TPW = (NT + NW - 1) / NW;              // n-tiles per wave (max)
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int i16 = lane & 15, kq = lane >> 4;
    s3_v4f acc[TPW];
    int tj[TPW][N - 1];
    bool tv[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        acc[q] = s3_v4f{0.f, 0.f, 0.f, 0.f};
        const int tau = 16 * (wv + NW * q) + i16;
        tv[q] = (wv + NW * q < NT) && tau < TAIL;
        int r = tv[q] ? tau : 0;
#pragma unroll
        for (int n = N - 2; n >= 0; --n) { tj[q][n] = r % JP; r /= JP; }
    }
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int t = k0 + kq;
        const float a = (i16 < JP) ? s_q[t * JP + i16] : 0.f;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (wv + NW * q < NT) {  // uniform over the wave
                float b = s_u[(t * (N - 1)) * JP + tj[q][0]];
#pragma unroll
                for (int n = 1; n < N - 1; ++n) b *= s_u[(t * (N - 1) + n) * JP + tj[q][n]];
                b = tv[q] ? b : 0.f;
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (!(wv + NW * q < NT)) continue;
        const int tau = 16 * (wv + NW * q) + i16;
        if (tau >= TAIL) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j1 = 4 * kq + r;
            if (j1 < JP) {
                float *c = core + (size_t)j1 * TAIL + tau;
                *c = add ? *c + acc[q][r] : acc[q][r];
            }
        }
    }
}

// Whether the det launch also forms each chunk's core-gradient partial (FP32
// Tucker cores on the matrix cores, hyper-diagonal cores on the VALU); an
// FP64 Tucker core takes k_core_partial after it.
template <typename T, int CT> constexpr bool det_fused_core() {
    return CT == kCP || std::is_same<T, float>::value;
}

// Whether the FP32 reuse contraction of a det block is split over its four
// wavefronts (64 entries per block; see det_tensor_split), and the entries per
// block and core chunk either way.
template <typename T, int CT> constexpr bool det_split() {
    return CT == kReuse && std::is_same<T, float>::value;
}
template <typename T, int CT> constexpr int det_chunk() { return det_split<T, CT>() ? kWave : kChunk; }

// Tensor entries of one det block, FP32 reuse contraction: the block's 64
// entries are contracted by all four wavefronts at once, wavefront w taking
// the core slices j1 = w, w + 4, ... (contract_part), so a batch spreads
// over four times as many wavefronts, each with a quarter of the serial
// work.  The partial w_2 .. w_N, x~, |w_1|^2 and |u^(1)|^2 meet in LDS and
// are added in wavefront order; wavefront w writes g_1 at its j1,
// wavefront n (1 <= n < N) the summed w_(n+1)'s row gradient g_(n+1) and
// curvature, wavefront 0 also L_1, q and L_G.  The rows then give the
// block's 64-entry core chunk on the matrix cores.  Same scratch row as the
// one-lane form below.
template <int N, int JP, bool ADJ>
S3_DEV void det_tensor_split(const TensorArgs<float> &A, const int32_t *__restrict__ ids, int64_t nt,
                             const float *__restrict__ Gp, float *__restrict__ scr, int64_t stride,
                             const float *__restrict__ gx, float *__restrict__ part, float *__restrict__ part_curv,
                             int64_t blk, const int32_t *__restrict__ bidx, const float *__restrict__ bval,
                             int64_t bstride) {
    using T = float;
    constexpr int S = kChunk / kWave, E = kWave, NI = (JP + S - 1) / S;
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    __shared__ float s_wp[S * (N - 1) * JP * E];  // [worker][mode - 2][k][entry]
    __shared__ float s_m[S * 3 * E];              // [worker][x~, |w_1|^2, |u^(1)|^2][entry]
    __shared__ float s_q[E * JP];
    __shared__ float s_u[E * (N - 1) * JP];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t s = blk * E + lane;
    const bool live = s < nt;
    T a[NI], v[N - 1][JP], w1[NI], wv[N - 1][JP];
    T xp = T(0), xv = T(0);
    int32_t rows[N];
    if (live) {
        // indices and value in item order (bidx/bval start at the batch's
        // first tensor item); the id is needed only for the adjoint's input
#pragma unroll
        for (int n = 0; n < N; ++n) rows[n] = bidx[(int64_t)n * bstride + s];
        const T *r0 = A.U[0] + (int64_t)rows[0] * A.J[0];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int j1 = w + S * i;
            a[i] = (j1 < A.J[0]) ? r0[j1] : T(0);
        }
#pragma unroll
        for (int n = 1; n < N; ++n) {
            const T *r = A.U[n] + (int64_t)rows[n] * A.J[n];
#pragma unroll
            for (int k = 0; k < JP; ++k) v[n - 1][k] = (k < A.J[n]) ? r[k] : T(0);
        }
        xv = ADJ ? gx[ids[s]] : bval[s];
        contract_part<N, JP, S, T>(Gp, w, a, v, w1, wv, xp);
    } else {
#pragma unroll
        for (int i = 0; i < NI; ++i) a[i] = w1[i] = T(0);
#pragma unroll
        for (int n = 0; n < N - 1; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) v[n][k] = wv[n][k] = T(0);
#pragma unroll
        for (int n = 0; n < N; ++n) rows[n] = 0;
    }
    T w1sq = T(0), a2 = T(0);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        w1sq = fmaT(w1[i], w1[i], w1sq);
        a2 = fmaT(a[i], a[i], a2);
    }
#pragma unroll
    for (int n = 0; n < N - 1; ++n)
#pragma unroll
        for (int k = 0; k < JP; ++k) s_wp[((w * (N - 1) + n) * JP + k) * E + lane] = wv[n][k];
    s_m[(w * 3 + 0) * E + lane] = xp;
    s_m[(w * 3 + 1) * E + lane] = w1sq;
    s_m[(w * 3 + 2) * E + lane] = a2;
    __syncthreads();
    T xhat = s_m[lane];
#pragma unroll
    for (int x = 1; x < S; ++x) xhat += s_m[x * 3 * E + lane];
    const T q = ADJ ? xv : -(xv - xhat);
    T curv = T(0);
    if (live) {
        T *out = scr + s * stride;
        const T reg0 = ADJ ? T(0) : A.lambda_reg / (T)A.cnt[0][rows[0]];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int j1 = w + S * i;
            if (j1 < JP) out[j1] = fmaT(q, w1[i], reg0 * a[i]);
        }
#pragma unroll
        for (int n = 1; n < N; ++n) {
            if (w != n) continue;  // uniform
            const T regn = ADJ ? T(0) : A.lambda_reg / (T)A.cnt[n][rows[n]];
            T ww = T(0);
#pragma unroll
            for (int k = 0; k < JP; ++k) {
                T t = s_wp[((n - 1) * JP + k) * E + lane];
#pragma unroll
                for (int x = 1; x < S; ++x) t += s_wp[((x * (N - 1) + n - 1) * JP + k) * E + lane];
                out[n * JP + k] = fmaT(q, t, regn * v[n - 1][k]);
                ww = fmaT(t, t, ww);
            }
            out[N * JP + n] = ww + regn;
        }
        if (w == 0) {
            T l1 = s_m[E + lane], uu0 = s_m[2 * E + lane];
#pragma unroll
            for (int x = 1; x < S; ++x) {
                l1 += s_m[(x * 3 + 1) * E + lane];
                uu0 += s_m[(x * 3 + 2) * E + lane];
            }
            out[N * JP] = l1 + reg0;
            curv = uu0;
#pragma unroll
            for (int n = 1; n < N; ++n) {
                T uu = T(0);
#pragma unroll
                for (int k = 0; k < JP; ++k) uu = fmaT(v[n - 1][k], v[n - 1][k], uu);
                curv *= uu;
            }
            out[stride - 2] = q;
            out[stride - 1] = curv;
        }
    }
    // the chunk's curvature sum, and its core gradient on the matrix cores
    if (w == 0) {
        curv = wave_sum(curv);
        if (lane == 0) part_curv[blk] = curv;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int j1 = w + S * i;
        if (j1 < JP) s_q[lane * JP + j1] = q * a[i];
    }
#pragma unroll
    for (int n = 1; n < N; ++n) {
        if (w != n) continue;  // uniform
#pragma unroll
        for (int k = 0; k < JP; ++k) s_u[(lane * (N - 1) + n - 1) * JP + k] = v[n - 1][k];
    }
    __syncthreads();
    core_tile_mfma<N, JP, E>(s_q, s_u, part + blk * (JP * TAIL));
}

// The one-lane form (FP64, the naive ablation and the hyper-diagonal core):
// block blk = entries [256 blk, 256 blk + 256) = core chunk blk.
template <int N, int JP, typename T, bool ADJ, int CT>
S3_DEV void det_tensor_lane(const TensorArgs<T> &A, const int32_t *__restrict__ ids, int64_t nt,
                            const T *__restrict__ Gp, T *__restrict__ scr, int64_t stride,
                            const T *__restrict__ gx, T *__restrict__ part, T *__restrict__ part_curv,
                            int64_t blk) {
    constexpr bool kFuse = det_fused_core<T, CT>();
    constexpr bool kMfma = kFuse && CT != kCP && !det_split<T, CT>();
    __shared__ float s_q[kMfma ? kChunk * JP : 1];
    __shared__ float s_u[kMfma ? kChunk * (N - 1) * JP : 1];
    __shared__ T s_red[kChunk / kWave][(kFuse && !kMfma) ? JP + 1 : 1];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t s = blk * kChunk + tid;
    T u[N][JP];
    T q = T(0), curv = T(0);
    if (s < nt) {
        const int64_t e = ids[s];
        T w[N][JP];
        int32_t rows[N];
        load_rows<N, JP, T>(A, e, u, rows);
        const T xv = ADJ ? gx[e] : A.val[e];
        T xhat;
        contract_any<CT, N, JP, T>(Gp, u, w, xhat);
        constexpr bool train = !ADJ;
        q = train ? -(xv - xhat) : xv;
        // fixed JP stride per mode (padding lanes hold zeros): stores at
        // run-time offsets here also make the compiler spill the core loads
        T *out = scr + s * stride;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T reg = train ? A.lambda_reg / (T)A.cnt[n][rows[n]] : T(0);
            T ww = T(0);
#pragma unroll
            for (int k = 0; k < JP; ++k) {
                out[n * JP + k] = fmaT(q, w[n][k], reg * u[n][k]);
                ww = fmaT(w[n][k], w[n][k], ww);
            }
            out[N * JP + n] = ww + reg;
        }
        curv = core_curv<CT, N, JP, T>(u);
        out[stride - 2] = q;
        out[stride - 1] = curv;
    } else {
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) u[n][k] = T(0);
    }
    if constexpr (kMfma) {
        // stage q u^(1) and the tail rows, then the chunk's MFMA tile
#pragma unroll
        for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = q * u[0][k];
#pragma unroll
        for (int n = 1; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) s_u[(tid * (N - 1) + n - 1) * JP + k] = u[n][k];
        curv = wave_sum(curv);
        if (lane == 0) s_red[wv][0] = curv;
        __syncthreads();
        constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
        core_tile_mfma<N, JP>(s_q, s_u, (float *)part + blk * (JP * TAIL));
        if (tid == 0) {
            T c = T(0);
            for (int x = 0; x < kChunk / kWave; ++x) c += s_red[x][0];
            part_curv[blk] = c;
        }
    } else if constexpr (kFuse) {
        // hyper-diagonal core: lane t holds q_t prod_n u_n[r] for every r;
        // the chunk sums go through the wavefronts in order
#pragma unroll
        for (int r = 0; r < JP; ++r) {
            T p = q;
#pragma unroll
            for (int n = 0; n < N; ++n) p *= u[n][r];
            const T t = wave_sum(p);
            if (lane == 0) s_red[wv][r] = t;
        }
        {
            const T t = wave_sum(curv);
            if (lane == 0) s_red[wv][JP] = t;
        }
        __syncthreads();
        if (tid <= JP) {
            T t = T(0);
            for (int x = 0; x < kChunk / kWave; ++x) t += s_red[x][tid];
            if (tid < JP) part[blk * JP + tid] = t;
            else part_curv[blk] = t;
        }
    }
}

// Tensor entries of one det block with the dense part of the contraction on
// the matrix cores (mfma.hpp): 256 entries, one lane each, block blk = core
// chunk blk.  Each wavefront stages its 64 entries' rows in LDS, contracts
// them together and reads back x~ and w_n; the scratch row and the chunk's
// core-gradient partial are those of det_tensor_lane (core gradient on the
// FP32 or BF16 matrix cores, FP32 sums).
template <int N, int JP, bool ADJ, int CT>
S3_DEV void det_tensor_mx(const TensorArgs<float> &A, const int32_t *__restrict__ ids, int64_t nt,
                          const void *__restrict__ g_fmt, float *__restrict__ scr, int64_t stride,
                          const float *__restrict__ gx, float *__restrict__ part, float *__restrict__ part_curv,
                          int64_t blk) {
    using T = float;
    constexpr int OP = (CT == kMfma16) ? kOpBF16 : kOpF32;
    constexpr int SLOT = MfmaDims<N, JP>::SLOT;
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int SLOTS = kChunk * SLOT, QU = kChunk * JP + kChunk * (N - 1) * JP;
    __shared__ __align__(16) float s_buf[SLOTS > QU ? SLOTS : QU];
    __shared__ __align__(16) unsigned char s_g[mfma_core_bytes<N, JP, OP>()];
    __shared__ float s_red[kChunk / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    mfma_load_core<N, JP, OP>(g_fmt, s_g);
    const int64_t s = blk * kChunk + tid;
    const bool live = s < nt;
    T u[N][JP];
    int32_t rows[N];
    int64_t e = 0;
    if (live) {
        e = ids[s];
        load_rows<N, JP, T>(A, e, u, rows);
    } else {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            rows[n] = 0;
#pragma unroll
            for (int k = 0; k < JP; ++k) u[n][k] = T(0);
        }
    }
    T *slots = s_buf + (size_t)wv * kWave * SLOT;
    T *mine = slots + (size_t)lane * SLOT;
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int k = 0; k < JP; k += 4)
            *(s3_v4f_m *)(mine + n * JP + k) = s3_v4f_m{u[n][k], u[n][k + 1], u[n][k + 2], u[n][k + 3]};
    // the value (or upstream gradient) and the regularisers load during the
    // contraction
    constexpr bool train = !ADJ;
    T xv = T(0), regs[N];
#pragma unroll
    for (int n = 0; n < N; ++n) regs[n] = T(0);
    if (live) {
        xv = ADJ ? gx[e] : A.val[e];
#pragma unroll
        for (int n = 0; n < N; ++n) regs[n] = train ? A.lambda_reg / (T)A.cnt[n][rows[n]] : T(0);
    }
    __syncthreads();  // slots and the staged core
    mfma_contract_wave<N, JP, OP>(slots, s_g);
    wave_lds_sync();  // a wavefront reads back only its own slots
    T w[N][JP];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int k = 0; k < JP; k += 4) {
            const s3_v4f_m t = *(const s3_v4f_m *)(mine + n * JP + k);
            w[n][k] = t[0];
            w[n][k + 1] = t[1];
            w[n][k + 2] = t[2];
            w[n][k + 3] = t[3];
        }
    const T xhat = mine[N * JP];
    __syncthreads();  // s_buf is reused for the core-gradient operands
    T q = T(0), curv = T(0);
    if (live) {
        q = train ? -(xv - xhat) : xv;
        T *out = scr + s * stride;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T reg = regs[n];
            T ww = T(0);
#pragma unroll
            for (int k = 0; k < JP; ++k) {
                out[n * JP + k] = fmaT(q, w[n][k], reg * u[n][k]);
                ww = fmaT(w[n][k], w[n][k], ww);
            }
            out[N * JP + n] = ww + reg;
        }
        curv = core_curv<kReuse, N, JP, T>(u);
        out[stride - 2] = q;
        out[stride - 1] = curv;
    }
    curv = wave_sum(curv);
    if (lane == 0) s_red[wv] = curv;
    if constexpr (N == 4) {
        core_grad_mx4<OP>(q, u, s_buf, part + blk * (JP * TAIL));
    } else {
        T *s_q = s_buf;
        T *s_u = s_buf + kChunk * JP;
#pragma unroll
        for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = q * u[0][k];
#pragma unroll
        for (int n = 1; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) s_u[(tid * (N - 1) + n - 1) * JP + k] = u[n][k];
        __syncthreads();
        if constexpr (OP == kOpBF16) core_tile_mfma_bf16<N, JP, kChunk>(s_q, s_u, part + blk * (JP * TAIL), kChunk);
        else core_tile_mfma<N, JP>(s_q, s_u, part + blk * (JP * TAIL));
    }
    if (tid == 0) {
        T c = T(0);
        for (int x = 0; x < kChunk / kWave; ++x) c += s_red[x];
        part_curv[blk] = c;
    }
}

// One det batch's entries in one launch.  Blocks [0, t_blocks): the tensor
// entries, block b = core chunk b (64 entries contracted by the block's four
// wavefronts together for the FP32 reuse contraction, det_tensor_split; else
// 256 entries, one lane each, det_tensor_lane).  Each entry's N factor rows
// are gathered, the single pass over the core (contract.hpp) gives x~, e and
// w_n, and the entry's scratch row is written:
//   [ g_1 (JP) | ... | g_N (JP) | L_1 .. L_N | q | L_G ]   (stride N*JP + N + 2)
// where g_n = q w_n + (lambda_reg / cnt_n) u_n is the Eq (8) row gradient,
// q = -e (training) or the upstream sensitivity (adjoint), L_n = |w_n|^2 +
// lambda_reg / cnt_n and L_G the entry's core curvature.  With a fused core
// the rows still in registers then give the chunk's core-gradient partial
//   P[b][j] = sum_{t in chunk} q_t u^(1)_t[j_1] ... u^(N)_t[j_N]   (padded j)
// and the chunk's curvature sum, in a fixed order.  Blocks from t_blocks on:
// one lane per coupled-matrix entry.
// ADJ = false: training gradients; ADJ = true: adjoint (q = gx[e], no
// regulariser).  The mode is a template flag and the entry's value is loaded
// before the contraction: with a run-time choice between two loads after it
// the compiler front-loads every scalar core load and spills them.
// two waves per SIMD for the matrix-core form (its LDS allows two blocks per CU)
template <int CT> constexpr int det_min_waves() { return is_mx(CT) ? 2 : 1; }

template <int N, int JP, typename T, bool ADJ, int CT = kReuse>
__global__ __launch_bounds__(kChunk, det_min_waves<CT>()) void k_det_entries(TensorArgs<T> A, const int32_t *__restrict__ ids,
                                                        int64_t nt, int64_t t_blocks, const T *__restrict__ Gp,
                                                        T *__restrict__ scr, int64_t stride,
                                                        const T *__restrict__ gx, T *__restrict__ part,
                                                        T *__restrict__ part_curv, DetMatArgs<T> B,
                                                        const int32_t *__restrict__ bidx,
                                                        const T *__restrict__ bval, int64_t bstride,
                                                        const void *__restrict__ g_fmt) {
    const int64_t blk = blockIdx.x;
    const int tid = threadIdx.x;
    if (blk >= t_blocks) {
        int m = 0;
        for (int h = 1; h < B.M; ++h)
            if (blk >= B.m[h].b0) m = h;
        const DetMatrix<T> &d = B.m[m];
        const int64_t s = (blk - d.b0) * kChunk + tid;
        if (s < d.n) det_matrix_entry(d, s, B.lambda_m, B.lambda_reg);
        return;
    }
    if constexpr (is_mx(CT)) {
        if constexpr (mfma_shape<N, JP>() && std::is_same<T, float>::value)
            det_tensor_mx<N, JP, ADJ, CT>(A, ids, nt, g_fmt, scr, stride, gx, part, part_curv, blk);
    } else if constexpr (det_split<T, CT>())
        det_tensor_split<N, JP, ADJ>(A, ids, nt, Gp, scr, stride, gx, part, part_curv, blk, bidx, bval, bstride);
    else
        det_tensor_lane<N, JP, T, ADJ, CT>(A, ids, nt, Gp, scr, stride, gx, part, part_curv, blk);
}

// ---------------------------------------------------------- det: core grad

// FP64 Tucker core-gradient partial over one chunk of kChunk entries of the
// batch (same sum as the fused FP32 tile, on the VALU):
//   P[chunk][j] = sum_{t in chunk} q_t u^(1)_t[j_1] ... u^(N)_t[j_N]   (padded j)
// Thread tau owns one index of modes 2..N and all JP values of mode 1.
template <int N, int JP, typename T>
__global__ __launch_bounds__(512) void k_core_partial(TensorArgs<T> A, const int32_t *__restrict__ ids,
                                                      int64_t nt, const T *__restrict__ scr,
                                                      int64_t stride, T *__restrict__ part,
                                                      T *__restrict__ part_curv) {
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int SUB = 64;
    __shared__ T s_q[SUB][JP];        // q_t * u^(1)_t
    __shared__ T s_u[SUB][N - 1][JP]; // tail rows
    __shared__ T s_curv[SUB];
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    const int64_t c1 = (c0 + kChunk < nt) ? c0 + kChunk : nt;
    int tj[N - 1];
    {
        int r = tid;
#pragma unroll
        for (int n = N - 2; n >= 0; --n) { tj[n] = r % JP; r /= JP; }
    }
    T acc[JP];
#pragma unroll
    for (int k = 0; k < JP; ++k) acc[k] = T(0);
    T curv = T(0);
    for (int64_t b0 = c0; b0 < c1; b0 += SUB) {
        const int cnt = (int)((c1 - b0 < SUB) ? c1 - b0 : SUB);
        __syncthreads();
        for (int x = tid; x < SUB * N; x += blockDim.x) {
            const int t = x / N, n = x % N;
            if (t < cnt) {
                const int64_t s = b0 + t;
                const int64_t e = ids[s];
                const int64_t row = A.idx[(int64_t)n * A.nnz + e];
                const T *r = A.U[n] + row * A.J[n];
                const T q = scr[s * stride + stride - 2];
#pragma unroll
                for (int k = 0; k < JP; ++k) {
                    const T v = (k < A.J[n]) ? r[k] : T(0);
                    if (n == 0) s_q[t][k] = q * v;
                    else s_u[t][n - 1][k] = v;
                }
                if (n == 0) s_curv[t] = scr[s * stride + stride - 1];
            }
        }
        __syncthreads();
        if (tid < TAIL) {
            for (int t = 0; t < cnt; ++t) {
                T p = s_u[t][0][tj[0]];
#pragma unroll
                for (int n = 1; n < N - 1; ++n) p *= s_u[t][n][tj[n]];
#pragma unroll
                for (int k = 0; k < JP; ++k) acc[k] = fmaT(s_q[t][k], p, acc[k]);
            }
        }
        if (tid == 0)
            for (int t = 0; t < cnt; ++t) curv += s_curv[t];
    }
    if (tid < TAIL) {
        T *o = part + (int64_t)blockIdx.x * (JP * TAIL);
#pragma unroll
        for (int k = 0; k < JP; ++k) o[k * TAIL + tid] = acc[k];
    }
    if (tid == 0) part_curv[blockIdx.x] = curv;
}

// The batch's core step, run by the last blocks of k_rows_reduce:
// G[j] -= eta * step, step = (sum_chunks P + nt * reg_core * G) / damp, and
// the padded copy Gp the next batch contracts with takes the new value;
// accumulate != 0: dG[j] += sum_chunks P (adjoint, Gp untouched).  One block
// per 16 padded core elements: lane el of phase ph sums chunks ph, ph + 16,
// ... of element el (and of the curvature), then the phases are added in
// order.  A hyper-diagonal core is one padded vector (Nc = 1).
template <typename T> struct CoreStep {
    T *G;                       // core, or its gradient in the adjoint
    T *Gp;                      // zero-padded JP^Nc copy (training only)
    const T *part, *part_curv;  // chunk partials [nchunks][KP], [nchunks]
    int64_t nchunks, nt, KP, blocks;
    int Nc, JP, Js[kMaxN];
    T reg_core, eta, kappa;
    int damp, accumulate;
};

template <typename T>
S3_DEV void core_step_block(const CoreStep<T> &c, int64_t blk, T (&s_p)[2][16][17]) {
    const int el = threadIdx.x & 15, ph = threadIdx.x >> 4;
    const int64_t KP = c.KP, nchunks = c.nchunks;
    const int64_t pj = blk * 16 + el;
    const int64_t pr = pj < KP ? pj : 0;
    T s0 = T(0), s1 = T(0), L0 = T(0), L1 = T(0);
    int64_t ch = ph;
    for (; ch + 16 < nchunks; ch += 32) {
        s0 += c.part[ch * KP + pr];
        s1 += c.part[(ch + 16) * KP + pr];
        L0 += c.part_curv[ch];
        L1 += c.part_curv[ch + 16];
    }
    for (; ch < nchunks; ch += 16) {
        s0 += c.part[ch * KP + pr];
        L0 += c.part_curv[ch];
    }
    s_p[0][ph][el] = s0 + s1;
    s_p[1][ph][el] = L0 + L1;
    __syncthreads();
    if (ph != 0 || pj >= KP) return;
    T s = T(0), L = T(0);
    for (int x = 0; x < 16; ++x) {
        s += s_p[0][x][el];
        L += s_p[1][x][el];
    }
    // padded index -> core index (the padding has no element)
    int64_t rem = pj, j = 0, mul = 1;
    for (int n = c.Nc - 1; n >= 0; --n) {
        const int jn = (int)(rem % c.JP);
        rem /= c.JP;
        if (jn >= c.Js[n]) return;
        j += jn * mul;
        mul *= c.Js[n];
    }
    if (c.accumulate) {
        c.G[j] += s;
    } else {
        const T g = s + (T)c.nt * c.reg_core * c.G[j];
        T scale = c.eta;
        if (c.damp) {
            const T d = c.kappa * c.eta * (L + (T)c.nt * c.reg_core);
            scale = c.eta / (d > T(1) ? d : T(1));
        }
        const T v = c.G[j] - scale * g;
        c.G[j] = v;
        c.Gp[pj] = v;
    }
}

// ---------------------------------------------------------- det: rows apply

// Each touched row of a batch is a segment of the row-sorted contribution
// list; its contributions (gradient row and curvature in the batch scratch)
// are summed in a fixed order and applied once.  Segment lengths follow the
// power law of the data, so three shapes share one launch:
//   lane blocks   one lane per segment of <= kShortSeg contributions (most
//                 rows), summed serially;
//   wave blocks   one wavefront per segment of up to kLongSeg (bind-time
//                 list): lanes stride the list, then a fixed butterfly;
//   piece blocks  the longer segments cut into pieces of kPiece
//                 contributions (bind-time list), one workgroup each (two
//                 contributions per lane, both loads in flight), whose
//                 sums k_rows_finish adds in piece order and applies (a
//                 single head row would otherwise run on one CU).
// All groups (factor matrices and coupled factors) of the batch go in the
// same two launches.  The thresholds are the fastest of a sweep on the
// 10M-entry Zipf(1.2) workload (batches of 65,536).
constexpr int64_t kShortSeg = 8;
constexpr int64_t kLongSeg = 128;
constexpr int64_t kPiece = 512;
constexpr int kRowsThreads = 256;
constexpr int kRowsJ = 16;  // largest rank

struct RowsGroup {
    const uint64_t *contrib;    // sorted (gradient offset | curvature offset << 32)
    const int64_t *seg_start;   // [nseg + 1]
    const int32_t *seg_row;
    const int32_t *med_ids;     // segments of (kShortSeg, kLongSeg] contributions
    const int32_t *long_ids;    // longer segments
    const int32_t *long_fp;     // first piece of each long segment (+ end)
    const int64_t *pc0, *pc1;   // pieces: contribution ranges
    void *P;                    // parameter (or gradient in the adjoint)
    int J;
    int64_t s0, s1, m0, m1, l0, l1, p0, p1;  // this batch's ranges
    int64_t b_lane, b_med, b_piece;          // first block of each kind
};

template <typename T> struct RowsArgs {
    RowsGroup g[kMaxN + kMaxM];
    int G;
    int64_t b_end;              // row blocks of k_rows_reduce
    int64_t n_long;             // long segments of the batch over all groups
    const T *scr;
    T *part;                    // piece sums [piece][kRowsJ + 1], pieces numbered across groups
    int64_t part_base[kMaxN + kMaxM];
    T eta, kappa;
    int damp, accumulate;
    CoreStep<T> core;           // blocks [b_end, b_end + core.blocks)
};

template <typename T>
S3_DEV void rows_update(T *P, int32_t row, int J, int k, T g, T L, const RowsArgs<T> &a) {
    T *p = P + (int64_t)row * J + k;
    if (a.accumulate) {
        *p += g;
    } else {
        T scale = a.eta;
        if (a.damp) {
            const T d = a.kappa * a.eta * L;
            scale = a.eta / (d > T(1) ? d : T(1));
        }
        *p -= scale * g;
    }
}

template <typename T>
__global__ __launch_bounds__(kRowsThreads) void k_rows_reduce(RowsArgs<T> a) {
    __shared__ T s_red[kRowsThreads / kWave][kRowsJ + 1];
    __shared__ T s_p[2][16][17];
    const int64_t blk = blockIdx.x;
    if (blk >= a.b_end) {
        core_step_block(a.core, blk - a.b_end, s_p);
        return;
    }
    int gi = 0;
    for (int h = 1; h < a.G; ++h)
        if (blk >= a.g[h].b_lane) gi = h;
    const RowsGroup &g = a.g[gi];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int J = g.J;
    if (blk < g.b_med) {
        // one lane per short segment
        const int64_t s = g.s0 + (blk - g.b_lane) * kRowsThreads + tid;
        if (s >= g.s1) return;
        const int64_t c0 = g.seg_start[s], c1 = g.seg_start[s + 1];
        if (c1 - c0 > kShortSeg) return;
        T acc[kRowsJ];
#pragma unroll
        for (int k = 0; k < kRowsJ; ++k) acc[k] = T(0);
        T L = T(0);
        // every contribution index first, then the rows four at a time with
        // predicated loads (all four in flight), added in contribution order
        uint64_t v[kShortSeg];
#pragma unroll
        for (int i = 0; i < kShortSeg; ++i) v[i] = (c0 + i < c1) ? g.contrib[c0 + i] : 0;
        constexpr int kGrp = 4;
#pragma unroll
        for (int h = 0; h < kShortSeg; h += kGrp) {
            if (c0 + h >= c1) break;
            T r[kGrp][kRowsJ], l[kGrp];
#pragma unroll
            for (int i = 0; i < kGrp; ++i) {
                const bool ok = c0 + h + i < c1;
                const T *gr = a.scr + (int64_t)(v[h + i] & 0xffffffffull);
#pragma unroll
                for (int k = 0; k < kRowsJ; ++k) r[i][k] = (ok && k < J) ? gr[k] : T(0);
                l[i] = ok ? a.scr[(int64_t)(v[h + i] >> 32)] : T(0);
            }
#pragma unroll
            for (int i = 0; i < kGrp; ++i) {
#pragma unroll
                for (int k = 0; k < kRowsJ; ++k)
                    if (k < J) acc[k] += r[i][k];
                L += l[i];
            }
        }
        const int32_t row = g.seg_row[s];
#pragma unroll
        for (int k = 0; k < kRowsJ; ++k)
            if (k < J) rows_update((T *)g.P, row, J, k, acc[k], L, a);
        return;
    }
    if (blk < g.b_piece) {
        // one wavefront per medium segment
        const int64_t m = g.m0 + (blk - g.b_med) * (kRowsThreads / kWave) + wv;
        if (m >= g.m1) return;  // uniform over the wavefront
        const int64_t s = g.med_ids[m];
        const int64_t c0 = g.seg_start[s], c1 = g.seg_start[s + 1];
        T acc[kRowsJ];
#pragma unroll
        for (int k = 0; k < kRowsJ; ++k) acc[k] = T(0);
        T L = T(0);
        int64_t c = c0 + lane;
        for (; c + kWave < c1; c += 2 * kWave) {
            const uint64_t v0 = g.contrib[c], v1 = g.contrib[c + kWave];
            const T *g0 = a.scr + (int64_t)(v0 & 0xffffffffull);
            const T *g1 = a.scr + (int64_t)(v1 & 0xffffffffull);
#pragma unroll
            for (int k = 0; k < kRowsJ; ++k)
                if (k < J) acc[k] += g0[k] + g1[k];
            L += a.scr[(int64_t)(v0 >> 32)] + a.scr[(int64_t)(v1 >> 32)];
        }
        if (c < c1) {
            const uint64_t v = g.contrib[c];
            const T *gr = a.scr + (int64_t)(v & 0xffffffffull);
#pragma unroll
            for (int k = 0; k < kRowsJ; ++k)
                if (k < J) acc[k] += gr[k];
            L += a.scr[(int64_t)(v >> 32)];
        }
        T mine = T(0);
#pragma unroll
        for (int k = 0; k < kRowsJ; ++k) {
            if (k >= J) break;  // uniform
            const T t = wave_sum(acc[k]);
            if (lane == k) mine = t;
        }
        L = wave_sum(L);
        if (lane < J) rows_update((T *)g.P, g.seg_row[s], J, lane, mine, L, a);
        return;
    }
    // one workgroup per piece of a long segment
    const int64_t pc = g.p0 + (blk - g.b_piece);
    const int64_t c0 = g.pc0[pc], c1 = g.pc1[pc];
    T acc[kRowsJ + 1];
#pragma unroll
    for (int k = 0; k <= kRowsJ; ++k) acc[k] = T(0);
    int64_t c = c0 + tid;
    for (; c + kRowsThreads < c1; c += 2 * kRowsThreads) {
        const uint64_t v0 = g.contrib[c], v1 = g.contrib[c + kRowsThreads];
        const T *g0 = a.scr + (int64_t)(v0 & 0xffffffffull);
        const T *g1 = a.scr + (int64_t)(v1 & 0xffffffffull);
#pragma unroll
        for (int k = 0; k < kRowsJ; ++k)
            if (k < J) acc[k] += g0[k] + g1[k];
        acc[kRowsJ] += a.scr[(int64_t)(v0 >> 32)] + a.scr[(int64_t)(v1 >> 32)];
    }
    if (c < c1) {
        const uint64_t v = g.contrib[c];
        const T *gr = a.scr + (int64_t)(v & 0xffffffffull);
#pragma unroll
        for (int k = 0; k < kRowsJ; ++k)
            if (k < J) acc[k] += gr[k];
        acc[kRowsJ] += a.scr[(int64_t)(v >> 32)];
    }
#pragma unroll
    for (int k = 0; k <= kRowsJ; ++k) {
        const T t = wave_sum(acc[k]);
        if (lane == 0) s_red[wv][k] = t;
    }
    __syncthreads();
    if (tid <= kRowsJ) {
        T t = T(0);
        for (int w = 0; w < kRowsThreads / kWave; ++w) t += s_red[w][tid];
        a.part[(a.part_base[gi] + pc - g.p0) * (kRowsJ + 1) + tid] = t;
    }
}

// one wavefront per long segment (over all groups): its pieces in order
template <typename T>
__global__ __launch_bounds__(kRowsThreads) void k_rows_finish(RowsArgs<T> a) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t w = ((int64_t)blockIdx.x * kRowsThreads + threadIdx.x) / kWave;
    if (w >= a.n_long) return;
    int gi = 0;
    for (; gi < a.G; ++gi) {
        const int64_t nl = a.g[gi].l1 - a.g[gi].l0;
        if (w < nl) break;
        w -= nl;
    }
    const RowsGroup &g = a.g[gi];
    const int64_t li = g.l0 + w;
    const int J = g.J;
    if (lane > J) return;
    // the pieces in order, four loads in flight
    const T *pp = a.part + (a.part_base[gi] - g.p0) * (kRowsJ + 1) + (lane < J ? lane : kRowsJ);
    const int64_t q1 = g.long_fp[li + 1];
    int64_t pc = g.long_fp[li];
    T t = T(0);
    for (; pc + 3 < q1; pc += 4) {
        const T x0 = pp[pc * (kRowsJ + 1)], x1 = pp[(pc + 1) * (kRowsJ + 1)];
        const T x2 = pp[(pc + 2) * (kRowsJ + 1)], x3 = pp[(pc + 3) * (kRowsJ + 1)];
        t += x0;
        t += x1;
        t += x2;
        t += x3;
    }
    for (; pc < q1; ++pc) t += pp[pc * (kRowsJ + 1)];
    const T L = __shfl(t, J, kWave);
    if (lane < J) rows_update((T *)g.P, g.seg_row[g.long_ids[li]], J, lane, t, L, a);
}

// bind time: the segments with lo < length <= hi, in order, with their batch
static __global__ void k_seg_class(const int64_t *__restrict__ seg_start, int64_t nseg, int64_t lo, int64_t hi,
                            int32_t *__restrict__ flag) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; s < nseg; s += stride) {
        const int64_t len = seg_start[s + 1] - seg_start[s];
        flag[s] = (len > lo && len <= hi) ? 1 : 0;
    }
}

static __global__ void k_seg_list(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int64_t nseg,
                           const uint32_t *__restrict__ seg_batch, const int64_t *__restrict__ seg_start,
                           int32_t *__restrict__ ids, uint32_t *__restrict__ batch, int64_t *__restrict__ c0,
                           int64_t *__restrict__ c1) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; s < nseg; s += stride)
        if (flag[s]) {
            const int64_t i = pos[s] - 1;
            ids[i] = (int32_t)s;
            batch[i] = seg_batch[s];
            if (c0) {
                c0[i] = seg_start[s];
                c1[i] = seg_start[s + 1];
            }
        }
}

// ---------------------------------------------------------------- evaluation

// sum over entries of (x - x~)^2: one entry per thread, one double partial
// per block (the host adds the partials in block order: deterministic)
template <int N, int JP, typename T, int CT = kReuse>
__global__ __launch_bounds__(256) void k_sq_err_tensor(TensorArgs<T> A, const T *__restrict__ Gp,
                                                       double *__restrict__ part) {
    __shared__ double s[256];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (e < A.nnz) {
        T u[N][JP];
        int32_t rows[N];
        load_rows<N, JP, T>(A, e, u, rows);
        const T r = A.val[e] - predict_any<CT, N, JP, T>(Gp, u);
        acc = (double)r * (double)r;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

template <int N, int JP, typename T, int CT = kReuse>
__global__ __launch_bounds__(256) void k_predict(TensorArgs<T> A, const T *__restrict__ Gp,
                                                 T *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < A.nnz) {
        T u[N][JP];
        int32_t rows[N];
        load_rows<N, JP, T>(A, e, u, rows);
        out[e] = predict_any<CT, N, JP, T>(Gp, u);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_predict_matrix(const int32_t *__restrict__ row,
                                                        const int32_t *__restrict__ col, int64_t nnz,
                                                        const T *__restrict__ Uc, const T *__restrict__ V,
                                                        int J, T *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const T *u = Uc + (int64_t)row[e] * J;
        const T *v = V + (int64_t)col[e] * J;
        T yh = T(0);
        for (int k = 0; k < J; ++k) yh = fmaT(u[k], v[k], yh);
        out[e] = yh;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sq_err_matrix(const int32_t *__restrict__ row,
                                                       const int32_t *__restrict__ col,
                                                       const T *__restrict__ val, int64_t nnz,
                                                       const T *__restrict__ Uc, const T *__restrict__ V,
                                                       int J, double *__restrict__ part) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const T *u = Uc + (int64_t)row[e] * J;
        const T *v = V + (int64_t)col[e] * J;
        T yh = T(0);
        for (int k = 0; k < J; ++k) yh = fmaT(u[k], v[k], yh);
        const T r = val[e] - yh;
        acc += (double)r * (double)r;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// sum over rows with cnt > 0 (all rows if cnt == null) of |row|^2
template <typename T>
__global__ __launch_bounds__(256) void k_sq_rows(const T *__restrict__ P, int64_t rows, int J,
                                                 const int32_t *__restrict__ cnt,
                                                 double *__restrict__ part) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (cnt && cnt[i] == 0) continue;
        const T *r = P + i * J;
        for (int k = 0; k < J; ++k) acc += (double)r[k] * (double)r[k];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// SplitMix64's output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014; the mixing constants of
// Vigna's splitmix64): a bijective mix of a 64-bit counter.
S3_DEV uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// n values N(0, sigma^2) from a counter-based generator: pair i takes the
// 53-bit uniforms of counters key + 2i and key + 2i + 1 (u1 in (0, 1], u2 in
// [0, 1)) through the Box-Muller transform, in FP64: elements 2i and 2i + 1
// are sigma sqrt(-2 ln u1) times cos and sin of 2 pi u2.
template <typename T>
__global__ void k_init_normal(T *__restrict__ p, int64_t n, uint64_t key, double sigma) {
    const int64_t pairs = (n + 1) / 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64_mix(key + 2 * (uint64_t)i);
        const uint64_t b = splitmix64_mix(key + 2 * (uint64_t)i + 1);
        const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;
        const double u2 = (double)(b >> 11) * 0x1.0p-53;
        const double r = sigma * sqrt(-2.0 * log(u1));
        const double t = 6.283185307179586 * u2;
        p[2 * i] = (T)(r * cos(t));
        if (2 * i + 1 < n) p[2 * i + 1] = (T)(r * sin(t));
    }
}

template <typename T>
__global__ void k_to_f64(const T *__restrict__ src, double *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

}  // namespace s3
