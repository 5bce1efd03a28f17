// Lock-free parallel SGD mode (Section 3.3 of the paper, re-designed for a
// GPU with tens of thousands of entries in flight).
//
// An epoch is a sequence of rounds; a round takes a slice of 256-entry
// tiles (tensor and coupled-matrix tiles, in a per-epoch shuffled tile
// order) and runs:
//   k_lf_tensor / k_lf_matrix  one workgroup per tile, one lane per entry;
//          each lane reads the current factor rows without locks, and for
//          each row it moves:
//            cold row -> at once, u <- u - eta g / max(1, k eta L) written
//                        back with plain stores (HOGWILD!-style: no lock, a
//                        concurrent write to the same row may win; a row
//                        touched by one entry of the round moves exactly like
//                        one SGD step)
//            hot row  -> gradient and curvature summed in an LDS table of
//                        the workgroup
//          the tile's core gradient is summed in registers (LDS-staged
//          operands); at the end the workgroup writes its whole hot-row
//          table and core partial to its own slot of a partials buffer
//          (plain coalesced stores: no global atomics).
//   k_lf_core_sum  sums the round's core partials in a fixed order.
//   k_lf_apply  one workgroup per hot row (and per core chunk): sums the
//          hot-row partials of every workgroup of the round in a fixed order
//          and moves the row / the core once by the damped step
//          -eta sum g / max(1, k eta sum L).
// "Hot" rows are the H most frequent rows of each mode and of each coupled
// factor.  The paper lets one worker own the core, which every entry
// touches; power-law data (a handful of rows in 10-30 % of all entries)
// needs the same treatment for its head rows, or thousands of concurrent
// stale updates of one row overshoot.
#pragma once
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace s3 {

constexpr int kTile = 256;

template <typename T> struct LFArgs {
    const int32_t *hot_slot[kMaxN + kMaxM];  // row -> slot in [0, H) or -1
    T *tab_out;        // per-workgroup hot tables: [wg][groups][H][JP + 1]
    T *core_out;       // per-workgroup core partials: [wg][KP + 2] (tensor only)
    int H;
    int JP;
    int64_t n_tiles;   // tiles of this kind
    int64_t tile_base; // first (permuted) tile index of this round
    uint64_t pa, pb;   // tile permutation i -> (pa * i + pb) mod n_tiles
};

S3_DEV int64_t lf_perm(int64_t i, uint64_t pa, uint64_t pb, int64_t n) {
    return (int64_t)((pa * (uint64_t)i + pb) % (uint64_t)n);  // pa, i < 2^31
}

// mode-1 slices per core-gradient work item: enough items for a 256-thread
// tile when the tail is short, and a divisor of JP
template <int JP, int TAIL> constexpr int lf_split() {
    int best = 1;
    for (int s = 1; s <= JP; ++s)
        if (JP % s == 0 && TAIL * s <= kTile) best = s;
    return best;
}

// ------------------------------------------------------------------ tensor

template <int N, int JP, typename T>
__global__ __launch_bounds__(kTile) void k_lf_tensor(TensorArgs<T> A, const T *__restrict__ Gp, LFArgs<T> L,
                                                     T eta, T kappa) {
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int KP = JP * TAIL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *s_tab = (T *)smem_raw;                         // [N][H][JP + 1]
    T *s_q = s_tab + (size_t)N * L.H * (JP + 1);     // [kTile][JP]  q * u^(1)
    T *s_u = s_q + kTile * JP;                        // [kTile][N - 1][JP]
    T *s_misc = s_u + (size_t)kTile * (N - 1) * JP;   // [0] core curvature, [1] count
    const int tid = threadIdx.x;
    const int tabn = N * L.H * (JP + 1);
    for (int i = tid; i < tabn; i += kTile) s_tab[i] = T(0);
    if (tid < 2) s_misc[tid] = T(0);
    __syncthreads();

    const int64_t tile = lf_perm(L.tile_base + blockIdx.x, L.pa, L.pb, L.n_tiles);
    const int64_t e = tile * kTile + tid;
    if (e < A.nnz) {
        T u[N][JP], w[N][JP];
        int32_t rows[N];
        load_rows<N, JP, T>(A, e, u, rows);
        const T xv = A.val[e];
        T xhat;
        contract<N, JP, T>(Gp, u, w, xhat);
        const T q = -(xv - xhat);
        T LG = T(1);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T reg = A.lambda_reg / (T)A.cnt[n][rows[n]];
            T ww = T(0), uu = T(0);
#pragma unroll
            for (int k = 0; k < JP; ++k) {
                ww = fmaT(w[n][k], w[n][k], ww);
                uu = fmaT(u[n][k], u[n][k], uu);
            }
            LG *= uu;
            const T ell = ww + reg;
            const int slot = L.hot_slot[n][rows[n]];
            if (slot >= 0) {
                T *t = s_tab + ((size_t)n * L.H + slot) * (JP + 1);
#pragma unroll
                for (int k = 0; k < JP; ++k) atomicAdd(&t[k], fmaT(q, w[n][k], reg * u[n][k]));
                atomicAdd(&t[JP], ell);
            } else {
                const T d = kappa * eta * ell;
                const T step = eta / (d > T(1) ? d : T(1));
                T *r = A.U[n] + (int64_t)rows[n] * A.J[n];
#pragma unroll
                for (int k = 0; k < JP; ++k)
                    if (k < A.J[n]) r[k] = u[n][k] - step * fmaT(q, w[n][k], reg * u[n][k]);
            }
        }
        // stage the core-gradient operands
#pragma unroll
        for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = q * u[0][k];
#pragma unroll
        for (int n = 1; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) s_u[((size_t)tid * (N - 1) + (n - 1)) * JP + k] = u[n][k];
        atomicAdd(&s_misc[0], LG);
        atomicAdd(&s_misc[1], T(1));
    } else {
#pragma unroll
        for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = T(0);
#pragma unroll
        for (int n = 1; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) s_u[((size_t)tid * (N - 1) + (n - 1)) * JP + k] = T(0);
    }
    __syncthreads();
    // core gradient of this tile: work item = (tail index tau over modes
    // 2..N, slice of JS consecutive mode-1 indices); all threads take part
    constexpr int SPLIT = lf_split<JP, TAIL>();
    constexpr int JS = JP / SPLIT;
    T *core = L.core_out + (size_t)blockIdx.x * (KP + 2);
    for (int item = tid; item < TAIL * SPLIT; item += kTile) {
        const int tau = item % TAIL, j0 = (item / TAIL) * JS;
        int tj[N - 1];
        int r = tau;
#pragma unroll
        for (int n = N - 2; n >= 0; --n) { tj[n] = r % JP; r /= JP; }
        T acc[JS];
#pragma unroll
        for (int k = 0; k < JS; ++k) acc[k] = T(0);
        for (int t = 0; t < kTile; ++t) {
            T p = s_u[((size_t)t * (N - 1)) * JP + tj[0]];
#pragma unroll
            for (int n = 1; n < N - 1; ++n) p *= s_u[((size_t)t * (N - 1) + n) * JP + tj[n]];
#pragma unroll
            for (int k = 0; k < JS; ++k) acc[k] = fmaT(s_q[t * JP + j0 + k], p, acc[k]);
        }
#pragma unroll
        for (int k = 0; k < JS; ++k) core[(size_t)(j0 + k) * TAIL + tau] = acc[k];
    }
    if (tid == 0) {
        core[KP] = s_misc[0];
        core[KP + 1] = s_misc[1];
    }
    // the workgroup's hot-row table, written densely
    T *tab = L.tab_out + (size_t)blockIdx.x * tabn;
    for (int i = tid; i < tabn; i += kTile) tab[i] = s_tab[i];
}

// ------------------------------------------------------------------ matrix

template <typename T>
__global__ __launch_bounds__(kTile) void k_lf_matrix(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                                                    const T *__restrict__ val, int64_t nnz, T *__restrict__ Uc,
                                                    T *__restrict__ V, int J, const int32_t *__restrict__ cntV,
                                                    T lambda_m, T lambda_reg, LFArgs<T> L, int gu, int gv,
                                                    T eta, T kappa) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *s_tab = (T *)smem_raw;  // [2][H][JP + 1]: coupled-mode rows, then V rows
    const int JP = L.JP;
    const int tid = threadIdx.x;
    const int tabn = 2 * L.H * (JP + 1);
    for (int i = tid; i < tabn; i += kTile) s_tab[i] = T(0);
    __syncthreads();
    const int64_t tile = lf_perm(L.tile_base + blockIdx.x, L.pa, L.pb, L.n_tiles);
    const int64_t e = tile * kTile + tid;
    if (e < nnz) {
        T *u = Uc + (int64_t)row[e] * J;
        T *v = V + (int64_t)col[e] * J;
        T ur[16], vr[16];
        T yh = T(0), uu = T(0), vv = T(0);
        for (int k = 0; k < J; ++k) {
            ur[k] = u[k];
            vr[k] = v[k];
            yh = fmaT(ur[k], vr[k], yh);
            uu = fmaT(ur[k], ur[k], uu);
            vv = fmaT(vr[k], vr[k], vv);
        }
        const T q = -lambda_m * (val[e] - yh);
        const T rv = lambda_m * lambda_reg / (T)cntV[col[e]];
        const T Lu = lambda_m * vv, Lv = fmaT(lambda_m, uu, rv);
        const int su = L.hot_slot[gu][row[e]];
        const int sv = L.hot_slot[gv][col[e]];
        if (su >= 0) {
            T *t = s_tab + (size_t)su * (JP + 1);
            for (int k = 0; k < J; ++k) atomicAdd(&t[k], q * vr[k]);
            atomicAdd(&t[JP], Lu);
        } else {
            const T d = kappa * eta * Lu;
            const T step = eta / (d > T(1) ? d : T(1));
            for (int k = 0; k < J; ++k) u[k] = ur[k] - step * q * vr[k];
        }
        if (sv >= 0) {
            T *t = s_tab + ((size_t)L.H + sv) * (JP + 1);
            for (int k = 0; k < J; ++k) atomicAdd(&t[k], fmaT(q, ur[k], rv * vr[k]));
            atomicAdd(&t[JP], Lv);
        } else {
            const T d = kappa * eta * Lv;
            const T step = eta / (d > T(1) ? d : T(1));
            for (int k = 0; k < J; ++k) v[k] = vr[k] - step * fmaT(q, ur[k], rv * vr[k]);
        }
    }
    __syncthreads();
    T *tab = L.tab_out + (size_t)blockIdx.x * tabn;
    for (int i = tid; i < tabn; i += kTile) tab[i] = s_tab[i];
}

// ------------------------------------------------------------------- apply

// Sources of one hot-row group in the round's partials: the tensor tables
// (group g < N) and every matrix table whose u-side (c_m == g) or V-side
// (g == N + m) is that group.
struct LFApplyArgs {
    void *P[kMaxN + kMaxM];                 // parameter of each group
    const int32_t *hot_row[kMaxN + kMaxM];  // slot -> row (or -1)
    int J[kMaxN + kMaxM];
    int groups;
    int N, M;
    int mat_mode[kMaxM];
    const void *tab_t;                      // tensor tables [nwg_t][N][H][JP+1]
    int64_t nwg_t;
    const void *tab_m[kMaxM];               // matrix tables [nwg_m][2][H][JP+1]
    int64_t nwg_m[kMaxM];
    const void *core_t;                     // tensor core partials [nwg_t][KP+2]
    const void *core_sum;                   // their sum over the round [KP+2]
};

constexpr int kApplyThreads = 256;

// fixed-order tree sum over the block of n values per thread (n <= 17)
template <typename T> S3_DEV void lf_block_sum(T *vals, int n, T *s_red) {
    const int tid = threadIdx.x;
    for (int k = 0; k < n; ++k) s_red[k * kApplyThreads + tid] = vals[k];
    __syncthreads();
    for (int w = kApplyThreads / 2; w > 0; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < n; ++k) s_red[k * kApplyThreads + tid] += s_red[k * kApplyThreads + tid + w];
        __syncthreads();
    }
    for (int k = 0; k < n; ++k) vals[k] = s_red[k * kApplyThreads];
}

// Fixed-order sum of the round's per-workgroup core partials (and their
// curvature and entry count): 16 consecutive elements per block, 16
// workgroup phases per element, four independent running sums per thread.
template <typename T>
__global__ __launch_bounds__(256) void k_lf_core_sum(const T *__restrict__ core_t, int64_t nwg, int64_t cs,
                                                     T *__restrict__ core_sum) {
    __shared__ T s_part[16][17];
    const int el = threadIdx.x & 15, ph = threadIdx.x >> 4;
    const int64_t j = (int64_t)blockIdx.x * 16 + el;
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    if (j < cs) {
        int64_t b = ph;
        for (; b + 48 < nwg; b += 64) {
            a0 += core_t[b * cs + j];
            a1 += core_t[(b + 16) * cs + j];
            a2 += core_t[(b + 32) * cs + j];
            a3 += core_t[(b + 48) * cs + j];
        }
        for (; b < nwg; b += 16) a0 += core_t[b * cs + j];
    }
    s_part[ph][el] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (ph == 0 && j < cs) {
        T t = T(0);
        for (int q = 0; q < 16; ++q) t += s_part[q][el];
        core_sum[j] = t;
    }
}

// blocks [0, groups * H): one hot row each; blocks after: core chunks of
// kApplyThreads elements
template <int N, typename T>
__global__ __launch_bounds__(kApplyThreads) void k_lf_apply(LFApplyArgs a, int H, int JP, T *__restrict__ G,
                                                            T *__restrict__ Gp, int J0, int J1, int J2, int J3,
                                                            T reg_core, T eta, T kappa) {
    __shared__ T s_red[17 * kApplyThreads];
    const int tid = threadIdx.x;
    const int nrowblk = a.groups * H;
    if ((int)blockIdx.x < nrowblk) {
        const int g = blockIdx.x / H, slot = blockIdx.x % H;
        const int row = a.hot_row[g][slot];
        if (row < 0) return;  // uniform over the block
        T acc[17];
        for (int k = 0; k < 17; ++k) acc[k] = T(0);
        const size_t W = (size_t)JP + 1;
        if (g < N) {
            const T *src = (const T *)a.tab_t + ((size_t)g * H + slot) * W;
            const size_t stride = (size_t)N * H * W;
            for (int64_t b = tid; b < a.nwg_t; b += kApplyThreads)
                for (int k = 0; k <= JP; ++k) acc[k] += src[b * stride + k];
        }
        for (int m = 0; m < a.M; ++m) {
            int side = -1;
            if (g < N && a.mat_mode[m] == g) side = 0;
            if (g == N + m) side = 1;
            if (side < 0) continue;
            const T *src = (const T *)a.tab_m[m] + ((size_t)side * H + slot) * W;
            const size_t stride = (size_t)2 * H * W;
            for (int64_t b = tid; b < a.nwg_m[m]; b += kApplyThreads)
                for (int k = 0; k <= JP; ++k) acc[k] += src[b * stride + k];
        }
        lf_block_sum<T>(acc, JP + 1, s_red);
        const T Lsum = acc[JP];
        if (Lsum != T(0) && tid < a.J[g]) {
            const T d = kappa * eta * Lsum;
            const T step = eta / (d > T(1) ? d : T(1));
            T *p = (T *)a.P[g] + (int64_t)row * a.J[g];
            T gk = T(0);
            for (int k = 0; k < JP; ++k)
                if (k == tid) gk = acc[k];
            p[tid] -= step * gk;
        }
        return;
    }
    // core (the round's sums come from k_lf_core_sum)
    const int Js[4] = {J0, J1, J2, J3};
    int K = 1, KP = 1;
    for (int n = 0; n < N; ++n) { K *= Js[n]; KP *= JP; }
    const int j = (blockIdx.x - nrowblk) * kApplyThreads + tid;
    const T *cs = (const T *)a.core_sum;
    const T LG = cs[KP], cnt = cs[KP + 1];
    if (j >= K || cnt == T(0)) return;
    int rem = j, pj = 0, mul = 1;
    for (int n = N - 1; n >= 0; --n) {
        const int jn = rem % Js[n];
        rem /= Js[n];
        pj += jn * mul;
        mul *= JP;
    }
    const T Lsum = LG + cnt * reg_core;
    const T d = kappa * eta * Lsum;
    const T step = eta / (d > T(1) ? d : T(1));
    const T gnew = G[j] - step * (cs[pj] + cnt * reg_core * G[j]);
    G[j] = gnew;
    Gp[pj] = gnew;
}

// ------------------------------------------------------------------- state

struct LockFreeState {
    int N = 0, M = 0, H = 0, JP = 0;
    int64_t KP = 0;
    int64_t nX = 0, y_nnz[kMaxM] = {};
    int64_t n_items = 0, n_rounds = 0;
    int64_t t_tiles = 0, m_tiles[kMaxM] = {};
    int64_t max_t_wg = 0, max_m_wg[kMaxM] = {};
    int32_t *hot_slot[kMaxN + kMaxM] = {};
    int32_t *hot_row[kMaxN + kMaxM] = {};
    int64_t rows[kMaxN + kMaxM] = {};
    void *tab_t = nullptr, *core_t = nullptr, *core_sum = nullptr;
    void *tab_m[kMaxM] = {};
    uint64_t seed = 0;
    bool ready = false;
    // per-launch state for the tensor kernel (set by lockfree_epoch)
    uint64_t pa = 1, pb = 0;
    LFApplyArgs apply{};
    const int32_t *cntV[kMaxM] = {};
    s3_buffers b{};
};

constexpr size_t kLfLdsBudget = 64 * 1024;

// hot rows per group: the requested count (power of two, <= 256) or, for 0,
// the largest that lets the tensor kernel's LDS fit the budget (0: none fits)
inline int lf_hot_rows(int N, int JP, size_t tsize, int requested) {
    const size_t staging = ((size_t)kTile * N * JP + 2) * tsize;
    for (int H = 256; H >= 16; H /= 2)
        if ((requested <= 0 || H <= requested) && staging + (size_t)N * H * (JP + 1) * tsize <= kLfLdsBudget)
            return H;
    return 0;
}

template <typename T, typename C>
void lockfree_layout(LockFreeState &s, C &c, int N, int M, const s3_desc &d, int64_t x_nnz, const int64_t *y_nnz,
                     int64_t KP, int JP) {
    s.N = N;
    s.M = M;
    s.JP = JP;
    s.KP = KP;
    s.H = lf_hot_rows(N, JP, sizeof(T), d.hot_rows);
    const int H = std::max(s.H, 1);
    int64_t n_items = x_nnz;
    for (int m = 0; m < M; ++m) n_items += y_nnz[m];
    const int64_t R = std::max<int64_t>(1, (n_items + d.round_items - 1) / d.round_items);
    const int64_t tt = (x_nnz + kTile - 1) / kTile;
    s.max_t_wg = (tt + R - 1) / R + 1;
    for (int n = 0; n < N; ++n) {
        s.rows[n] = d.dims[n];
        s.hot_slot[n] = c.template take<int32_t>((size_t)d.dims[n]);
        s.hot_row[n] = c.template take<int32_t>((size_t)H);
    }
    for (int m = 0; m < M; ++m) {
        s.rows[N + m] = d.mat_cols[m];
        s.hot_slot[N + m] = c.template take<int32_t>((size_t)d.mat_cols[m]);
        s.hot_row[N + m] = c.template take<int32_t>((size_t)H);
        const int64_t mt = (y_nnz[m] + kTile - 1) / kTile;
        s.max_m_wg[m] = (mt + R - 1) / R + 1;
        s.tab_m[m] = c.template take<T>((size_t)s.max_m_wg[m] * 2 * H * (JP + 1));
    }
    s.tab_t = c.template take<T>((size_t)s.max_t_wg * N * H * (JP + 1));
    s.core_t = c.template take<T>((size_t)s.max_t_wg * (KP + 2));
    s.core_sum = c.template take<T>((size_t)KP + 2);
}

// pick the H most frequent rows of every group (host side, from the counts)
template <typename T>
s3_status lockfree_build(LockFreeState &s, const s3_desc &d, const s3_buffers *buf, int32_t *const *cnt,
                         int32_t *const *cntV, int64_t nX, const int64_t *y_nnz, hipStream_t st, std::string &err) {
    const int N = s.N, M = s.M;
    s.nX = nX;
    s.n_items = nX;
    s.b = *buf;
    for (int m = 0; m < M; ++m) {
        s.y_nnz[m] = y_nnz[m];
        s.n_items += y_nnz[m];
        s.cntV[m] = cntV[m];
    }
    s.seed = d.seed;
    s.n_rounds = std::max<int64_t>(1, (s.n_items + d.round_items - 1) / d.round_items);
    s.t_tiles = (nX + kTile - 1) / kTile;
    for (int m = 0; m < M; ++m) s.m_tiles[m] = (y_nnz[m] + kTile - 1) / kTile;
    if (s.H == 0) return S3_OK;  // lock-free mode unavailable; reported by s3_epoch
    for (int g = 0; g < N + M; ++g) {
        const int64_t R = s.rows[g];
        std::vector<int32_t> h((size_t)R);
        const int32_t *src = (g < N) ? cnt[g] : cntV[g - N];
        if (hipMemcpyAsync(h.data(), src, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            err = "copying counts to the host failed";
            return S3_ERR_HIP;
        }
        std::vector<int32_t> order((size_t)R);
        std::iota(order.begin(), order.end(), 0);
        const int64_t take = std::min<int64_t>(s.H, R);
        std::partial_sort(order.begin(), order.begin() + take, order.end(), [&](int32_t a, int32_t b) {
            return h[a] != h[b] ? h[a] > h[b] : a < b;
        });
        std::vector<int32_t> slot((size_t)R, -1), hr((size_t)s.H, -1);
        for (int64_t k = 0; k < take; ++k) {
            if (h[order[k]] == 0) break;
            slot[order[k]] = (int32_t)k;
            hr[k] = order[k];
        }
        if (hipMemcpyAsync(s.hot_slot[g], slot.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(s.hot_row[g], hr.data(), sizeof(int32_t) * s.H, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            err = "uploading the hot-row tables failed";
            return S3_ERR_HIP;
        }
        s.apply.hot_row[g] = s.hot_row[g];
        s.apply.P[g] = (g < N) ? buf->U[g] : buf->V[g - N];
        s.apply.J[g] = (g < N) ? d.rank[g] : d.rank[d.mat_mode[g - N]];
    }
    s.apply.groups = N + M;
    s.apply.N = N;
    s.apply.M = M;
    for (int m = 0; m < M; ++m) {
        s.apply.mat_mode[m] = d.mat_mode[m];
        s.apply.tab_m[m] = s.tab_m[m];
    }
    s.apply.tab_t = s.tab_t;
    s.apply.core_t = s.core_t;
    s.apply.core_sum = s.core_sum;
    s.ready = true;
    return S3_OK;
}

template <typename T> LFArgs<T> lf_args(const LockFreeState &s, int64_t n_tiles, int64_t base, T *tab, T *core) {
    LFArgs<T> L{};
    for (int g = 0; g < s.N + s.M; ++g) L.hot_slot[g] = s.hot_slot[g];
    L.tab_out = tab;
    L.core_out = core;
    L.H = s.H;
    L.JP = s.JP;
    L.n_tiles = n_tiles;
    L.tile_base = base;
    L.pa = s.pa;
    L.pb = s.pb;
    return L;
}

template <int N, int JP, typename T>
void lockfree_tensor_launch(LockFreeState &s, const TensorArgs<T> &A, const T *Gp, int64_t first, int64_t count,
                            T eta, hipStream_t st) {
    if (count <= 0) return;
    LFArgs<T> L = lf_args<T>(s, s.t_tiles, first, (T *)s.tab_t, (T *)s.core_t);
    const size_t smem = ((size_t)N * s.H * (JP + 1) + (size_t)kTile * JP * N + 2) * sizeof(T);
    hipLaunchKernelGGL((k_lf_tensor<N, JP, T>), dim3((unsigned)count), dim3(kTile), smem, st, A, Gp, L, eta,
                       (T)(N + 1));
}

inline uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

inline void pick_perm(uint64_t &rng, int64_t n, uint64_t &pa, uint64_t &pb) {
    if (n <= 1) { pa = 1; pb = 0; return; }
    for (;;) {
        uint64_t a = 1 + splitmix64(rng) % (uint64_t)(n - 1);
        if (std::gcd(a, (uint64_t)n) == 1) { pa = a; break; }
    }
    pb = splitmix64(rng) % (uint64_t)n;
}

// One lock-free epoch.  tensor_round(first_tile, count, eta, stream) launches
// the tensor kernel for one round; the caller padded the core into Gp.
template <typename T, typename F>
s3_status lockfree_epoch(LockFreeState &s, const s3_desc &d, int epoch, double eta, T *Gp, hipStream_t st,
                         std::string &err, F tensor_round) {
    if (!s.ready) { err = "lock-free tables not built"; return S3_ERR_STATE; }
    const int N = s.N, M = s.M;
    uint64_t rng = s.seed * 0x2545F4914F6CDD1Dull + (uint64_t)epoch * 0x9E3779B97F4A7C15ull + 1;
    uint64_t tpa, tpb, mpa[kMaxM], mpb[kMaxM];
    pick_perm(rng, s.t_tiles, tpa, tpb);
    for (int m = 0; m < M; ++m) pick_perm(rng, s.m_tiles[m], mpa[m], mpb[m]);
    const int64_t R = s.n_rounds;
    const T kappa = (T)(N + 1);
    const T reg_core = (T)(d.lambda_reg / (double)s.nX);
    const int *J = d.rank;
    int64_t K = 1;
    for (int n = 0; n < N; ++n) K *= J[n];
    for (int64_t r = 0; r < R; ++r) {
        const int64_t t0 = s.t_tiles * r / R, t1 = s.t_tiles * (r + 1) / R;
        s.pa = tpa;
        s.pb = tpb;
        tensor_round(t0, t1 - t0, eta, st);
        s.apply.nwg_t = t1 - t0;
        for (int m = 0; m < M; ++m) {
            const int64_t m0 = s.m_tiles[m] * r / R, m1 = s.m_tiles[m] * (r + 1) / R;
            s.apply.nwg_m[m] = std::max<int64_t>(0, m1 - m0);
            if (m1 <= m0) continue;
            s.pa = mpa[m];
            s.pb = mpb[m];
            LFArgs<T> L = lf_args<T>(s, s.m_tiles[m], m0, (T *)s.tab_m[m], nullptr);
            const int c = d.mat_mode[m];
            const size_t smem = (size_t)2 * s.H * (s.JP + 1) * sizeof(T);
            hipLaunchKernelGGL(k_lf_matrix<T>, dim3((unsigned)(m1 - m0)), dim3(kTile), smem, st, s.b.y_row[m],
                               s.b.y_col[m], (const T *)s.b.y_val[m], s.y_nnz[m], (T *)s.b.U[c], (T *)s.b.V[m],
                               J[c], s.cntV[m], (T)d.lambda_m, (T)d.lambda_reg, L, c, N + m, (T)eta, kappa);
        }
        if (t1 > t0)
            hipLaunchKernelGGL(k_lf_core_sum<T>, dim3((unsigned)((s.KP + 2 + 15) / 16)), dim3(256), 0, st,
                               (const T *)s.core_t, t1 - t0, s.KP + 2, (T *)s.core_sum);
        else
            hipLaunchKernelGGL(k_fill<T>, dim3(4), dim3(256), 0, st, (T *)s.core_sum, s.KP + 2, T(0));
        const int64_t blocks = (int64_t)(N + M) * s.H + (K + kApplyThreads - 1) / kApplyThreads;
        auto kern = (N == 3) ? k_lf_apply<3, T> : k_lf_apply<4, T>;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kApplyThreads), 0, st, s.apply, s.H, s.JP,
                           (T *)s.b.G, Gp, J[0], J[1], J[2], N > 3 ? J[3] : 1, reg_core, (T)eta, kappa);
    }
    return S3_OK;
}

}  // namespace s3
