// Lock-free parallel SGD mode (Section 3.3 of the paper, re-designed for a
// GPU with tens of thousands of entries in flight).
//
// An epoch is a sequence of rounds; a round takes a slice of 256-entry
// tiles (tensor and coupled-matrix tiles, in a per-epoch shuffled tile
// order) and runs three launches:
//   k_lf_tensor / k_lf_matrix  one lane per entry, reads the current
//          factor rows without locks; the row it moves:
//            cold row -> at once, atomic add of -eta g / max(1, k eta L)
//                        (HOGWILD!-style; a row touched by one entry of the
//                        round moves exactly like one SGD step)
//            hot row  -> gradient and curvature summed in an LDS table per
//                        workgroup, flushed to a global accumulator
//          and the core gradient is summed per workgroup (LDS staging)
//          into a global accumulator.
//   k_lf_apply  moves every hot row and the core once by the damped step
//          -eta sum g / max(1, k eta sum L) and clears the accumulators.
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
    T *acc;                                  // [(N + M)][H][JP + 1]
    T *accG;                                 // [KP] then [KP] = curvature, [KP+1] = entry count
    int H;
    int JP;
    int64_t n_tiles;   // tiles of this kind
    int64_t tile_base; // first (permuted) tile index of this round
    int64_t n_round;   // tiles in this round
    uint64_t pa, pb;   // tile permutation i -> (pa * i + pb) mod n_tiles
};

S3_DEV int64_t lf_perm(int64_t i, uint64_t pa, uint64_t pb, int64_t n) {
    return (int64_t)((pa * (uint64_t)i + pb) % (uint64_t)n);  // pa, i < 2^31
}

// ------------------------------------------------------------------ tensor

template <int N, int JP, typename T>
__global__ __launch_bounds__(kTile) void k_lf_tensor(TensorArgs<T> A, const T *__restrict__ Gp, LFArgs<T> L,
                                                     T eta, T kappa) {
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int SUB = 64;
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
    const bool live = e < A.nnz;
    T u[N][JP], w[N][JP];
    int32_t rows[N];
    if (live) {
        load_rows<N, JP, T>(A, e, u, rows);
        T xhat;
        contract<N, JP, T>(Gp, u, w, xhat);
        const T q = -(A.val[e] - xhat);
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
                for (int k = 0; k < JP; ++k)
                    if (k < A.J[n]) atomicAdd(&t[k], fmaT(q, w[n][k], reg * u[n][k]));
                atomicAdd(&t[JP], ell);
            } else {
                const T d = kappa * eta * ell;
                const T step = eta / (d > T(1) ? d : T(1));
                T *r = A.U[n] + (int64_t)rows[n] * A.J[n];
#pragma unroll
                for (int k = 0; k < JP; ++k)
                    if (k < A.J[n]) atomicAdd(&r[k], -step * fmaT(q, w[n][k], reg * u[n][k]));
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
    // core gradient of this tile: thread owns tail indices tau (modes 2..N)
    for (int tau = tid; tau < TAIL; tau += kTile) {
        int tj[N - 1];
        int r = tau;
#pragma unroll
        for (int n = N - 2; n >= 0; --n) { tj[n] = r % JP; r /= JP; }
        T acc[JP];
#pragma unroll
        for (int k = 0; k < JP; ++k) acc[k] = T(0);
        for (int t0 = 0; t0 < kTile; t0 += SUB) {
            for (int t = t0; t < t0 + SUB; ++t) {
                T p = s_u[((size_t)t * (N - 1)) * JP + tj[0]];
#pragma unroll
                for (int n = 1; n < N - 1; ++n) p *= s_u[((size_t)t * (N - 1) + n) * JP + tj[n]];
#pragma unroll
                for (int k = 0; k < JP; ++k) acc[k] = fmaT(s_q[t * JP + k], p, acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < JP; ++k) atomicAdd(&L.accG[(size_t)k * TAIL + tau], acc[k]);
    }
    if (tid == 0) {
        const int64_t KP = (int64_t)JP * TAIL;
        atomicAdd(&L.accG[KP], s_misc[0]);
        atomicAdd(&L.accG[KP + 1], s_misc[1]);
    }
    // flush touched hot rows
    for (int i = tid; i < N * L.H; i += kTile) {
        const T *t = s_tab + (size_t)i * (JP + 1);
        if (t[JP] != T(0)) {
            T *g = L.acc + (size_t)i * (JP + 1);
            for (int k = 0; k <= JP; ++k) atomicAdd(&g[k], t[k]);
        }
    }
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
    for (int i = tid; i < 2 * L.H * (JP + 1); i += kTile) s_tab[i] = T(0);
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
            for (int k = 0; k < J; ++k) atomicAdd(&u[k], -step * q * vr[k]);
        }
        if (sv >= 0) {
            T *t = s_tab + ((size_t)L.H + sv) * (JP + 1);
            for (int k = 0; k < J; ++k) atomicAdd(&t[k], fmaT(q, ur[k], rv * vr[k]));
            atomicAdd(&t[JP], Lv);
        } else {
            const T d = kappa * eta * Lv;
            const T step = eta / (d > T(1) ? d : T(1));
            for (int k = 0; k < J; ++k) atomicAdd(&v[k], -step * fmaT(q, ur[k], rv * vr[k]));
        }
    }
    __syncthreads();
    for (int i = tid; i < 2 * L.H; i += kTile) {
        const T *t = s_tab + (size_t)i * (JP + 1);
        if (t[JP] != T(0)) {
            const int g = (i < L.H) ? gu : gv;
            const int slot = (i < L.H) ? i : i - L.H;
            T *dst = L.acc + ((size_t)g * L.H + slot) * (JP + 1);
            for (int k = 0; k <= JP; ++k) atomicAdd(&dst[k], t[k]);
        }
    }
}

// ------------------------------------------------------------------- apply

struct LFApplyArgs {
    void *P[kMaxN + kMaxM];        // parameter of each group
    const int32_t *hot_row[kMaxN + kMaxM];  // slot -> row (or -1)
    int J[kMaxN + kMaxM];
    int groups;
};

template <int N, typename T>
__global__ void k_lf_apply(LFApplyArgs a, T *__restrict__ acc, int H, int JP, T *__restrict__ G,
                           T *__restrict__ Gp, T *__restrict__ accG, int J0, int J1, int J2, int J3,
                           T reg_core, T eta, T kappa) {
    const int Js[4] = {J0, J1, J2, J3};
    int K = 1, KP = 1;
    for (int n = 0; n < N; ++n) { K *= Js[n]; KP *= JP; }
    const int nrow = a.groups * H;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < nrow) {
        const int g = (int)(tid / H), slot = (int)(tid % H);
        T *t = acc + (size_t)tid * (JP + 1);
        const int row = a.hot_row[g][slot];
        const T Lsum = t[JP];
        if (row >= 0 && Lsum != T(0)) {
            const T d = kappa * eta * Lsum;
            const T step = eta / (d > T(1) ? d : T(1));
            T *p = (T *)a.P[g] + (int64_t)row * a.J[g];
            for (int k = 0; k < a.J[g]; ++k) p[k] -= step * t[k];
        }
        for (int k = 0; k <= JP; ++k) t[k] = T(0);
    } else if (tid < nrow + K) {
        const int j = (int)(tid - nrow);
        int rem = j, pj = 0, mul = 1;
        for (int n = N - 1; n >= 0; --n) {
            const int jn = rem % Js[n];
            rem /= Js[n];
            pj += jn * mul;
            mul *= JP;
        }
        const T cntT = accG[KP + 1];
        if (cntT != T(0)) {
            const T Lsum = accG[KP] + cntT * reg_core;
            const T d = kappa * eta * Lsum;
            const T step = eta / (d > T(1) ? d : T(1));
            const T gnew = G[j] - step * (accG[pj] + cntT * reg_core * G[j]);
            G[j] = gnew;
            Gp[pj] = gnew;
        }
    }
}

// clear the core accumulator (after every thread of k_lf_apply has read it)
template <typename T> __global__ void k_lf_clear(T *__restrict__ accG, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        accG[i] = T(0);
}

// ------------------------------------------------------------------- state

struct LockFreeState {
    int N = 0, M = 0, H = 0, JP = 0;
    int64_t KP = 0;
    int64_t nX = 0, y_nnz[kMaxM] = {};
    int64_t n_items = 0, n_rounds = 0;
    int64_t t_tiles = 0, m_tiles[kMaxM] = {};
    int32_t *hot_slot[kMaxN + kMaxM] = {};
    int32_t *hot_row[kMaxN + kMaxM] = {};
    int64_t rows[kMaxN + kMaxM] = {};
    void *acc = nullptr;
    void *accG = nullptr;
    uint64_t seed = 0;
    bool ready = false;
    // per-launch state for the tensor kernel (set by lockfree_epoch)
    uint64_t pa = 1, pb = 0;
    int64_t tile_base = 0, n_round = 0;
    LFApplyArgs apply{};
    int J[kMaxN] = {};
    double lambda_reg = 0, lambda_m = 0;
    const s3_buffers *buf = nullptr;
    s3_buffers b{};
    const int32_t *cntV[kMaxM] = {};
};

constexpr size_t kLfLdsBudget = 64 * 1024;

// hot rows per group so that the tensor kernel's LDS fits the budget (0: none fits)
inline int lf_hot_rows(int N, int JP, size_t tsize) {
    const size_t staging = ((size_t)kTile * N * JP + 2) * tsize;
    for (int H = 256; H >= 16; H /= 2)
        if (staging + (size_t)N * H * (JP + 1) * tsize <= kLfLdsBudget) return H;
    return 0;
}

template <typename T, typename C>
void lockfree_layout(LockFreeState &s, C &c, int N, int M, const s3_desc &d, int64_t x_nnz, const int64_t *y_nnz,
                     int64_t KP, int JP) {
    s.N = N;
    s.M = M;
    s.JP = JP;
    s.KP = KP;
    s.H = lf_hot_rows(N, JP, sizeof(T));
    for (int n = 0; n < N; ++n) {
        s.rows[n] = d.dims[n];
        s.hot_slot[n] = c.template take<int32_t>((size_t)d.dims[n]);
        s.hot_row[n] = c.template take<int32_t>((size_t)s.H);
    }
    for (int m = 0; m < M; ++m) {
        s.rows[N + m] = d.mat_cols[m];
        s.hot_slot[N + m] = c.template take<int32_t>((size_t)d.mat_cols[m]);
        s.hot_row[N + m] = c.template take<int32_t>((size_t)s.H);
    }
    s.acc = c.template take<T>((size_t)(N + M) * s.H * (JP + 1));
    s.accG = c.template take<T>((size_t)KP + 2);
    (void)x_nnz;
    (void)y_nnz;
}

// pick the H most frequent rows of every group (host side, from the counts)
template <typename T>
s3_status lockfree_build(LockFreeState &s, const s3_desc &d, const s3_buffers *buf, int32_t *const *cnt,
                         int32_t *const *cntV, int64_t nX, const int64_t *y_nnz, hipStream_t st, std::string &err) {
    const int N = s.N, M = s.M;
    s.nX = nX;
    s.n_items = nX;
    s.b = *buf;
    s.lambda_reg = d.lambda_reg;
    s.lambda_m = d.lambda_m;
    for (int m = 0; m < M; ++m) {
        s.y_nnz[m] = y_nnz[m];
        s.n_items += y_nnz[m];
        s.cntV[m] = cntV[m];
    }
    for (int n = 0; n < N; ++n) s.J[n] = d.rank[n];
    s.seed = d.seed;
    s.n_rounds = std::max<int64_t>(1, (s.n_items + d.round_items - 1) / d.round_items);
    s.t_tiles = (nX + kTile - 1) / kTile;
    for (int m = 0; m < M; ++m) s.m_tiles[m] = (y_nnz[m] + kTile - 1) / kTile;
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
    const int64_t nacc = (int64_t)(N + M) * s.H * (s.JP + 1);
    hipLaunchKernelGGL(k_fill<T>, dim3(64), dim3(256), 0, st, (T *)s.acc, nacc, T(0));
    hipLaunchKernelGGL(k_fill<T>, dim3(64), dim3(256), 0, st, (T *)s.accG, s.KP + 2, T(0));
    s.ready = true;
    return S3_OK;
}

template <typename T> LFArgs<T> lf_args(const LockFreeState &s, int64_t n_tiles, int64_t base, int64_t count) {
    LFArgs<T> L{};
    for (int g = 0; g < s.N + s.M; ++g) L.hot_slot[g] = s.hot_slot[g];
    L.acc = (T *)s.acc;
    L.accG = (T *)s.accG;
    L.H = s.H;
    L.JP = s.JP;
    L.n_tiles = n_tiles;
    L.tile_base = base;
    L.n_round = count;
    L.pa = s.pa;
    L.pb = s.pb;
    return L;
}

template <int N, int JP, typename T>
void lockfree_tensor_launch(LockFreeState &s, const TensorArgs<T> &A, const T *Gp, int64_t first, int64_t count,
                            T eta, hipStream_t st) {
    if (count <= 0) return;
    LFArgs<T> L = lf_args<T>(s, s.t_tiles, first, count);
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
// the tensor kernel for one round (the caller owns the core padding).
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
    const int64_t nrow = (int64_t)(N + M) * s.H;
    int64_t K = 1;
    for (int n = 0; n < N; ++n) K *= J[n];
    for (int64_t r = 0; r < R; ++r) {
        const int64_t t0 = s.t_tiles * r / R, t1 = s.t_tiles * (r + 1) / R;
        s.pa = tpa;
        s.pb = tpb;
        tensor_round(t0, t1 - t0, eta, st);
        for (int m = 0; m < M; ++m) {
            const int64_t m0 = s.m_tiles[m] * r / R, m1 = s.m_tiles[m] * (r + 1) / R;
            if (m1 <= m0) continue;
            s.pa = mpa[m];
            s.pb = mpb[m];
            LFArgs<T> L = lf_args<T>(s, s.m_tiles[m], m0, m1 - m0);
            const int c = d.mat_mode[m];
            const size_t smem = (size_t)2 * s.H * (s.JP + 1) * sizeof(T);
            hipLaunchKernelGGL(k_lf_matrix<T>, dim3((unsigned)(m1 - m0)), dim3(kTile), smem, st, s.b.y_row[m],
                               s.b.y_col[m], (const T *)s.b.y_val[m], s.y_nnz[m], (T *)s.b.U[c], (T *)s.b.V[m],
                               J[c], s.cntV[m], (T)d.lambda_m, (T)d.lambda_reg, L, c, N + m, (T)eta, kappa);
        }
        const int64_t nthreads = nrow + K;
        auto kern = (N == 3) ? k_lf_apply<3, T> : k_lf_apply<4, T>;
        hipLaunchKernelGGL(kern, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st, s.apply, (T *)s.acc,
                           s.H, s.JP, (T *)s.b.G, Gp, (T *)s.accG, J[0], J[1], J[2],
                           N > 3 ? J[3] : 1, reg_core, (T)eta, kappa);
        hipLaunchKernelGGL(k_lf_clear<T>, dim3(16), dim3(256), 0, st, (T *)s.accG, s.KP + 2);
    }
    return S3_OK;
}

}  // namespace s3
