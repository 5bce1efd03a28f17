// Lock-free parallel SGD mode (Section 3.3 of the paper, re-designed for a
// GPU with tens of thousands of entries in flight).
//
// An epoch is a sequence of rounds; a round takes a slice of 256-entry
// tiles (tensor and coupled-matrix tiles, in a per-epoch shuffled tile
// order) and runs:
//   k_lf_tensor  one workgroup per tile (tensor tiles, then the round's
//          coupled-matrix tiles in the same launch), one lane per entry;
//          each lane reads the current factor rows without locks, and for
//          each row it moves:
//            cold row -> at once, u <- u - eta g / max(1, k eta L) written
//                        back with plain stores (HOGWILD!-style: no lock, a
//                        concurrent write to the same row may win; a row
//                        touched by one entry of the round moves exactly like
//                        one SGD step)
//            hot row  -> gradient and curvature summed in an LDS table of
//                        the workgroup
//          the tile's core gradient is one small GEMM on the FP32 matrix
//          cores (LDS-staged operands); at the end the workgroup writes its
//          whole hot-row
//          table and core partial to its own slot of a partials buffer
//          (plain coalesced stores: no global atomics).
//   k_lf_tensor_mx  the same with the dense part of the contraction on the
//          matrix cores (mfma.hpp): persistent workgroups, each running
//          ceil(tiles / 512) of the round's tiles with the core's operand
//          image staged once and its hot table and core partial carried
//          from tile to tile; each tile's entry streams are loaded while the
//          tile before it runs.
//   k_lf_apply  one workgroup per hot row and one per 16 core elements:
//          sums the round's partials of every workgroup in a fixed order and
//          moves the row / the core once by the damped step
//          -eta sum g / max(1, k eta sum L); for matrix-core plans it also
//          rewrites the core values it changes in the operand image.
// "Hot" rows are the H most frequent rows of each mode and of each coupled
// factor.  The paper lets one worker own the core, which every entry
// touches; power-law data (a handful of rows in 10-30 % of all entries)
// needs the same treatment for its head rows, or thousands of concurrent
// stale updates of one row overshoot.
#pragma once
#include <hip/hip_ext.h>
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "mfma.hpp"

namespace s3 {

constexpr int kTile = 256;
constexpr int64_t kMxResident = 512;  // tensor workgroups of the matrix-core round kernel (2 per CU)

template <typename T> struct LFArgs {
    const int32_t *hot_slot[kMaxN + kMaxM];  // row -> slot in [0, H) or -1
    const uint2 *meta_slot;  // per tensor entry: sorted hot position per mode, int16 each (-1: cold)
    const uint32_t *chunks;  // [tile][N][kTile] chunk descriptors
    const int32_t *nchunks;  // [tile][N]
    const T *meta_reg;       // per tensor entry and mode: lambda_reg / |Omega^{n,i_n}|, [N][nnz]
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

// Hot-row contributions without atomics.  At bind time the hot entries of
// every 256-entry tile are sorted by slot, per group (tensor mode, or u / V
// side of a matrix); each entry keeps its position in that order and the
// sorted run is cut into chunks of at most 16 entries of one slot.  In a
// round an entry writes its gradient row (and curvature) to its position in
// LDS with plain stores; one work item per (chunk, element) then sums the
// chunk and stores it in the slot's table row (an atomic add only where a
// slot's run spans several chunks).  Chunk descriptor: slot (bits 0-7),
// first position (8-15), length - 1 (16-19), whole run (20).
constexpr int kRun = 16;

// per-entry packed int16 fields: slot (at bind) / position (after), -1 = cold
S3_DEV int lf_field(uint2 m, int g) {
    const uint32_t h = g < 2 ? m.x : m.y;
    return (int)(int16_t)((g & 1) ? (h >> 16) : (h & 0xffffu));
}
S3_DEV int lf_field(uint32_t m, int g) { return (int)(int16_t)((g & 1) ? (m >> 16) : (m & 0xffffu)); }
S3_DEV uint32_t lf_put(uint32_t h, int g, int v) {
    const uint32_t f = (uint32_t)(uint16_t)(int16_t)v;
    return (g & 1) ? ((h & 0xffffu) | (f << 16)) : ((h & 0xffff0000u) | f);
}
S3_DEV void lf_set(uint2 &m, int g, int v) {
    if (g < 2) m.x = lf_put(m.x, g, v); else m.y = lf_put(m.y, g, v);
}
S3_DEV void lf_set(uint32_t &m, int g, int v) { m = lf_put(m, g, v); }
template <typename P> S3_DEV P lf_cold();
template <> S3_DEV uint2 lf_cold<uint2>() { return make_uint2(0xffffffffu, 0xffffffffu); }
template <> S3_DEV uint32_t lf_cold<uint32_t>() { return 0xffffffffu; }

// G groups of one tile: s_stage [G][JP + 1][kTile] (sorted positions),
// s_tab [G][H][JP + 1] (zeroed); between two barriers
// ACC: the table already holds earlier tiles' sums (a workgroup that runs
// several tiles), so a whole run is added to it rather than stored.
// A thread takes work items tid, tid + kTile, ...; their chunk descriptors
// are loaded kChunkBatch at a time before any is used, so the global loads
// overlap instead of each waiting for the one before.
constexpr int kChunkBatch = 8;

template <int JP, int G, typename T, bool ACC = false>
S3_DEV void lf_chunk_pass(const T *s_stage, T *s_tab, const uint32_t *chunks, const int32_t *nchunks, int H) {
    constexpr int W = JP + 1;
    int base[G + 1];
    base[0] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) base[g + 1] = base[g] + nchunks[g] * W;
    for (int i0 = threadIdx.x; i0 < base[G]; i0 += kChunkBatch * kTile) {
        uint32_t d[kChunkBatch];
        int gk[kChunkBatch];  // group * W + element
#pragma unroll
        for (int b = 0; b < kChunkBatch; ++b) {
            const int item = i0 + b * kTile;
            d[b] = 0;
            gk[b] = 0;
            if (item < base[G]) {
                int g = 0;
#pragma unroll
                for (int h = 1; h < G; ++h) g += item >= base[h];
                const int c = (item - base[g]) / W, k = (item - base[g]) - c * W;
                d[b] = chunks[(size_t)g * kTile + c];
                gk[b] = g * W + k;
            }
        }
#pragma unroll
        for (int b = 0; b < kChunkBatch; ++b) {
            if (i0 + b * kTile >= base[G]) break;
            const int g = gk[b] / W, k = gk[b] - g * W;
            const int slot = d[b] & 0xff, start = (d[b] >> 8) & 0xff, len = ((d[b] >> 16) & 0xf) + 1;
            const T *src = s_stage + (size_t)gk[b] * kTile + start;
            T sum = T(0);
#pragma unroll
            for (int j = 0; j < kRun; ++j)
                if (j < len) sum += src[j];
            T *dst = s_tab + ((size_t)g * H + slot) * W + k;
            if ((d[b] >> 20) & 1) {
                if constexpr (ACC) *dst += sum;
                else *dst = sum;
            } else {
                atomicAdd(dst, sum);
            }
        }
    }
}

// bind time: slots -> positions and chunk descriptors, one workgroup per tile
template <typename P, int G>
__global__ __launch_bounds__(kTile) void k_lf_chunks(P *__restrict__ meta, int64_t nnz, uint32_t *__restrict__ chunks,
                                                     int32_t *__restrict__ nchunks) {
    __shared__ int s_slot[kTile];
    __shared__ int s_wtot[kTile / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int64_t tile = blockIdx.x;
    const int64_t e = tile * kTile + tid;
    P m = (e < nnz) ? meta[e] : lf_cold<P>();
    for (int g = 0; g < G; ++g) {
        const int slot = lf_field(m, g);
        s_slot[tid] = slot;
        __syncthreads();
        int pos = 0, seg0 = 0, seglen = 0;
        if (slot >= 0)
            for (int l = 0; l < kTile; ++l) {
                const int s2 = s_slot[l];
                const bool lower = s2 >= 0 && s2 < slot;
                seg0 += lower;
                seglen += s2 == slot;
                pos += lower || (s2 == slot && l < tid);
            }
        const bool head = slot >= 0 && (pos - seg0) % kRun == 0;
        const uint64_t bal = __ballot(head);
        if (lane == 0) s_wtot[wv] = __popcll(bal);
        __syncthreads();
        int cidx = __popcll(bal & ((1ull << lane) - 1)), total = 0;
        for (int w = 0; w < kTile / kWave; ++w) {
            if (w < wv) cidx += s_wtot[w];
            total += s_wtot[w];
        }
        if (head) {
            const int len = min(kRun, seg0 + seglen - pos);
            chunks[((size_t)tile * G + g) * kTile + cidx] = (uint32_t)slot | ((uint32_t)pos << 8) |
                                                            ((uint32_t)(len - 1) << 16) |
                                                            ((seglen <= kRun ? 1u : 0u) << 20);
        }
        if (tid == 0) nchunks[tile * G + g] = total;
        lf_set(m, g, slot >= 0 ? pos : -1);
        __syncthreads();
    }
    if (e < nnz) meta[e] = m;
}

// ------------------------------------------------------------------ matrix

// Coupled-matrix tiles of one round; they run in the same launch as the
// tensor tiles (blocks after the tensor blocks), in matrix order.
template <typename T> struct LFMatArgs {
    const int32_t *row[kMaxM];
    const int32_t *col[kMaxM];
    const T *val[kMaxM];
    int64_t nnz[kMaxM];
    T *Uc[kMaxM];
    T *V[kMaxM];
    int J[kMaxM];
    const int32_t *cntV[kMaxM];
    int64_t n_tiles[kMaxM];   // tiles of the matrix
    int64_t tile_base[kMaxM]; // first permuted tile of this round
    int64_t n_blocks[kMaxM];  // tiles of this round
    uint64_t pa[kMaxM], pb[kMaxM];
    T *tab_out[kMaxM];        // [wg][2][H][JP + 1]
    const uint32_t *meta_slot[kMaxM];  // per entry: u-side and V-side sorted hot positions (int16, -1 cold)
    const uint32_t *chunks[kMaxM];     // [tile][2][kTile]
    const int32_t *nchunks[kMaxM];     // [tile][2]
    const T *meta_rv[kMaxM];           // per entry: lambda_m lambda_reg / |Omega_Y^{2,k}|
    int gu[kMaxM], gv[kMaxM];
    int M;
    T lambda_m;
};

template <int JP, typename T, bool EXACT>
S3_DEV void lf_matrix_tile(const LFMatArgs<T> &Y, int m, int64_t blk, const LFArgs<T> &L, T eta, T kappa,
                           T *s_tab) {
    constexpr int W = JP + 1;
    const int tid = threadIdx.x;
    const int tabn = 2 * L.H * W;
    T *s_stage = s_tab + tabn;  // [2][W][kTile]
    for (int i = tid; i < tabn; i += kTile) s_tab[i] = T(0);
    const int64_t tile = lf_perm(Y.tile_base[m] + blk, Y.pa[m], Y.pb[m], Y.n_tiles[m]);
    const int64_t e = tile * kTile + tid;
    const int J = EXACT ? JP : Y.J[m];
    if (e < Y.nnz[m]) {
        const int32_t r = Y.row[m][e], cl = Y.col[m][e];
        const uint32_t ms = Y.meta_slot[m][e];
        T *u = Y.Uc[m] + (int64_t)r * J;
        T *v = Y.V[m] + (int64_t)cl * J;
        T ur[JP], vr[JP];
        T yh = T(0), uu = T(0), vv = T(0);
#pragma unroll
        for (int k = 0; k < JP; ++k) {
            ur[k] = (EXACT || k < J) ? u[k] : T(0);
            vr[k] = (EXACT || k < J) ? v[k] : T(0);
            yh = fmaT(ur[k], vr[k], yh);
            uu = fmaT(ur[k], ur[k], uu);
            vv = fmaT(vr[k], vr[k], vv);
        }
        const T q = -Y.lambda_m * (Y.val[m][e] - yh);
        const T rv = Y.meta_rv[m][e];
        const T Lu = Y.lambda_m * vv, Lv = fmaT(Y.lambda_m, uu, rv);
        const int pu = lf_field(ms, 0), pv = lf_field(ms, 1);
        if (pu >= 0) {
            T *t = s_stage + pu;
#pragma unroll
            for (int k = 0; k < JP; ++k) t[k * kTile] = q * vr[k];
            t[JP * kTile] = Lu;
        } else {
            const T d = kappa * eta * Lu;
            const T step = eta / (d > T(1) ? d : T(1));
#pragma unroll
            for (int k = 0; k < JP; ++k)
                if (EXACT || k < J) u[k] = ur[k] - step * q * vr[k];
        }
        if (pv >= 0) {
            T *t = s_stage + W * kTile + pv;
#pragma unroll
            for (int k = 0; k < JP; ++k) t[k * kTile] = fmaT(q, ur[k], rv * vr[k]);
            t[JP * kTile] = Lv;
        } else {
            const T d = kappa * eta * Lv;
            const T step = eta / (d > T(1) ? d : T(1));
#pragma unroll
            for (int k = 0; k < JP; ++k)
                if (EXACT || k < J) v[k] = vr[k] - step * fmaT(q, ur[k], rv * vr[k]);
        }
    }
    __syncthreads();
    lf_chunk_pass<JP, 2>(s_stage, s_tab, Y.chunks[m] + (size_t)tile * 2 * kTile, Y.nchunks[m] + tile * 2, L.H);
    __syncthreads();
    T *tab = Y.tab_out[m] + (size_t)blk * tabn;
    for (int i = tid; i < tabn; i += kTile) tab[i] = s_tab[i];
}

// ------------------------------------------------------------------ tensor

// Blocks [0, n_tensor): tensor tiles.  Blocks after: the round's matrix
// tiles, matrix by matrix.
// minimum waves per SIMD requested from the register allocator: 3 for cores
// of up to 1,024 entries (fits in 168 VGPRs without spilling, and matches the
// three 256-thread workgroups per CU the LDS allows), 1 otherwise
template <int N, int JP, int CT = kReuse> constexpr int lf_min_waves() {
    return (CT == kCP || (N == 3 ? JP * JP * JP : JP * JP * JP * JP) <= 1024) ? 3 : 1;
}

template <int N, int JP, typename T, bool EXACT, int CT = kReuse>
__global__ __launch_bounds__(kTile, (lf_min_waves<N, JP, CT>())) void k_lf_tensor(TensorArgs<T> A, const T *__restrict__ Gp,
                                                                          LFArgs<T> L, LFMatArgs<T> Y,
                                                                          int64_t n_tensor, T eta, T kappa) {
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int KP = (CT == kCP) ? JP : JP * TAIL;  // stored core values (padded)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if ((int64_t)blockIdx.x >= n_tensor) {
        int64_t blk = (int64_t)blockIdx.x - n_tensor;
        for (int m = 0; m < Y.M; ++m) {
            if (blk < Y.n_blocks[m]) {
                lf_matrix_tile<JP, T, EXACT>(Y, m, blk, L, eta, kappa, (T *)smem_raw);
                return;
            }
            blk -= Y.n_blocks[m];
        }
        return;
    }
    constexpr int W = JP + 1;
    constexpr int NWV = kTile / kWave;
    T *s_tab = (T *)smem_raw;                         // [N][H][W]
    T *s_misc = s_tab + (size_t)N * L.H * W;          // per wavefront: core curvature, entry count
    T *s_stage = s_misc + 2 * NWV;                    // [N][W][kTile] sorted hot rows, then:
    T *s_q = s_stage;                                 // [kTile][JP]  q * u^(1)
    T *s_u = s_q + kTile * JP;                        // [kTile][N - 1][JP]
    const int tid = threadIdx.x;
    const int tabn = N * L.H * W;
    for (int i = tid; i < tabn; i += kTile) s_tab[i] = T(0);

    const int64_t tile = lf_perm(L.tile_base + blockIdx.x, L.pa, L.pb, L.n_tiles);
    const int64_t e = tile * kTile + tid;
    const bool live = e < A.nnz;
    T u[N][JP];
    T q = T(0), LG = T(0);
    if (live) {
        T w[N][JP];
        int32_t rows[N];
        load_rows<N, JP, T, EXACT>(A, e, u, rows);
        const T xv = A.val[e];
        const uint2 ms = L.meta_slot[e];
        T regs[N];
#pragma unroll
        for (int n = 0; n < N; ++n) regs[n] = L.meta_reg[(int64_t)n * A.nnz + e];
        T xhat;
        contract_any<CT, N, JP, T>(Gp, u, w, xhat);
        q = -(xv - xhat);
        LG = T(1);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T reg = regs[n];
            T ww = T(0), uu = T(0);
#pragma unroll
            for (int k = 0; k < JP; ++k) {
                ww = fmaT(w[n][k], w[n][k], ww);
                uu = fmaT(u[n][k], u[n][k], uu);
            }
            LG *= uu;
            const T ell = ww + reg;
            const int pos = lf_field(ms, n);
            if (pos >= 0) {
                T *t = s_stage + (size_t)n * W * kTile + pos;
#pragma unroll
                for (int k = 0; k < JP; ++k) t[k * kTile] = fmaT(q, w[n][k], reg * u[n][k]);
                t[JP * kTile] = ell;
            } else {
                const T d = kappa * eta * ell;
                const T step = eta / (d > T(1) ? d : T(1));
                T *r = A.U[n] + (int64_t)rows[n] * (EXACT ? JP : A.J[n]);
#pragma unroll
                for (int k = 0; k < JP; ++k)
                    if (EXACT || k < A.J[n]) r[k] = u[n][k] - step * fmaT(q, w[n][k], reg * u[n][k]);
            }
        }
        if constexpr (CT == kCP) LG = core_curv<kCP, N, JP, T>(u);
    }
    {
        const T lg = wave_sum(LG);
        const uint64_t bal = __ballot(live);
        if ((tid & (kWave - 1)) == 0) {
            s_misc[2 * (tid / kWave)] = lg;
            s_misc[2 * (tid / kWave) + 1] = (T)__popcll(bal);
        }
    }
    __syncthreads();
    lf_chunk_pass<JP, N>(s_stage, s_tab, L.chunks + (size_t)tile * N * kTile, L.nchunks + tile * N, L.H);
    __syncthreads();
    T *core = L.core_out + (size_t)blockIdx.x * (KP + 2);
    if constexpr (CT == kCP) {
        // hyper-diagonal core: lane sums of q prod_n u_n[r], added over the
        // wavefronts in order (the sorted rows are consumed, so s_stage is free)
        T *s_red = s_stage;  // [NWV][JP]
        T c[JP];
#pragma unroll
        for (int r = 0; r < JP; ++r) c[r] = T(0);
        if (live) {
#pragma unroll
            for (int r = 0; r < JP; ++r) {
                T p = q;
#pragma unroll
                for (int n = 0; n < N; ++n) p *= u[n][r];
                c[r] = p;
            }
        }
#pragma unroll
        for (int r = 0; r < JP; ++r) {
            const T t = wave_sum(c[r]);
            if ((tid & (kWave - 1)) == 0) s_red[(tid / kWave) * JP + r] = t;
        }
        __syncthreads();
        if (tid < JP) {
            T t = T(0);
            for (int w = 0; w < NWV; ++w) t += s_red[w * JP + tid];
            core[tid] = t;
        }
    } else {
    // stage the core-gradient operands (over the sorted rows, now consumed)
    if (live) {
#pragma unroll
        for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = q * u[0][k];
#pragma unroll
        for (int n = 1; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) s_u[((size_t)tid * (N - 1) + (n - 1)) * JP + k] = u[n][k];
    } else {
#pragma unroll
        for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = T(0);
#pragma unroll
        for (int n = 1; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; ++k) s_u[((size_t)tid * (N - 1) + (n - 1)) * JP + k] = T(0);
    }
    __syncthreads();
    if constexpr (std::is_same<T, float>::value) {
        core_tile_mfma<N, JP>(s_q, s_u, core);
    } else {
        // core gradient of this tile on the VALU: work item = (tail index tau
        // over modes 2..N, slice of JS consecutive mode-1 indices)
        constexpr int SPLIT = lf_split<JP, TAIL>();
        constexpr int JS = JP / SPLIT;
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
    }
    }  // Tucker core
    if (tid == 0) {
        T lg = T(0), cnt = T(0);
        for (int w = 0; w < NWV; ++w) {
            lg += s_misc[2 * w];
            cnt += s_misc[2 * w + 1];
        }
        core[KP] = lg;
        core[KP + 1] = cnt;
    }
    // the workgroup's hot-row table, written densely
    __syncthreads();
    T *tab = L.tab_out + (size_t)blockIdx.x * tabn;
    for (int i = tid; i < tabn; i += kTile) tab[i] = s_tab[i];
}

// The same round kernel with the dense part of every entry's contraction
// on the matrix cores (mfma.hpp).  A tensor workgroup runs several of the
// round's tiles in turn (tiles b, b + n_tensor, ...): the core's operands are
// staged in LDS once, and the hot-row tables, the core-gradient sums and the
// curvature sums carry over from tile to tile, so each workgroup writes one
// table and one core partial per round.  Per tile, each wavefront stages its
// 64 entries' rows, contracts them together and reads back x~ and w_n; the
// per-entry updates, hot-row sums and the matrix tiles (one per workgroup, in
// the blocks after the tensor ones) are those of k_lf_tensor.  The core
// gradient runs on the FP32 or BF16 matrix cores, summed in FP32.  FP32
// parameters (the master copies).
// One lane's entry stream of a tensor tile in a round (see k_lf_tensor_mx)
template <int N, typename T> struct LfStream {
    int32_t idx[N];
    T reg[N];
    T xv;
    uint2 ms;
};

template <int N, typename T>
S3_DEV void lf_fetch_stream(const TensorArgs<T> &A, const LFArgs<T> &L, int64_t it, LfStream<N, T> &s, int64_t &e,
                            bool &live) {
    const int64_t tile = lf_perm(L.tile_base + it, L.pa, L.pb, L.n_tiles);
    e = tile * kTile + threadIdx.x;
    live = e < A.nnz;
    if (live) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            s.idx[n] = A.idx[(int64_t)n * A.nnz + e];
            s.reg[n] = L.meta_reg[(int64_t)n * A.nnz + e];
        }
        s.xv = A.val[e];
        s.ms = L.meta_slot[e];
    }
}

template <int N, int JP, bool EXACT, int CT>
__global__ __launch_bounds__(kTile, 2) void k_lf_tensor_mx(TensorArgs<float> A, const void *__restrict__ g_fmt,
                                                           LFArgs<float> L, LFMatArgs<float> Y, int64_t n_tensor,
                                                           int64_t n_tiles, float eta, float kappa) {
    using T = float;
    constexpr int OP = (CT == kMfma16) ? kOpBF16 : kOpF32;
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int KP = JP * TAIL;
    constexpr int SLOT = MfmaDims<N, JP>::SLOT;
    constexpr int GB = mfma_core_bytes<N, JP, OP>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if ((int64_t)blockIdx.x >= n_tensor) {
        int64_t blk = (int64_t)blockIdx.x - n_tensor;
        for (int m = 0; m < Y.M; ++m) {
            if (blk < Y.n_blocks[m]) {
                lf_matrix_tile<JP, T, EXACT>(Y, m, blk, L, eta, kappa, (T *)smem_raw);
                return;
            }
            blk -= Y.n_blocks[m];
        }
        return;
    }
    constexpr int W = JP + 1;
    constexpr int NWV = kTile / kWave;
    void *s_g = smem_raw;                              // staged core operands
    T *s_tab = (T *)(smem_raw + GB);                   // [N][H][W]
    T *s_misc = s_tab + (size_t)N * L.H * W;
    T *s_stage = s_misc + 4 * ((2 * NWV + 3) / 4);     // 16-byte aligned; [N][W][kTile] sorted hot rows,
                                                       // before that the entry slots, after it the
                                                       // core-gradient operands
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int tabn = N * L.H * W;
    for (int i = tid; i < tabn; i += kTile) s_tab[i] = T(0);
    mfma_load_core<N, JP, OP>(g_fmt, s_g);
    T *core = L.core_out + (size_t)blockIdx.x * (KP + 2);
    s3_v16f cacc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    T lg_tot = T(0), cnt_tot = T(0);  // thread 0: curvature and entry counts of its tiles
    bool first = true;

    // A tile's entry streams (mode indices, value, hot positions,
    // regularisers) are loaded while the tile before it is processed, so at a
    // tile's start only its row gathers wait on memory.
    LfStream<N, T> cs;
    int64_t e = 0;
    bool live = false;
    lf_fetch_stream<N, T>(A, L, blockIdx.x, cs, e, live);

#pragma unroll 1
    for (int64_t it = blockIdx.x; it < n_tiles; it += n_tensor) {  // uniform over the block
        const int64_t tile = lf_perm(L.tile_base + it, L.pa, L.pb, L.n_tiles);
        T u[N][JP];
        int32_t rows[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            rows[n] = live ? cs.idx[n] : 0;
            const T *r = A.U[n] + (int64_t)rows[n] * (EXACT ? JP : A.J[n]);
#pragma unroll
            for (int k = 0; k < JP; ++k) u[n][k] = (live && (EXACT || k < A.J[n])) ? r[k] : T(0);
        }
        const bool more = it + n_tensor < n_tiles;
        LfStream<N, T> ns;
        int64_t ne = 0;
        bool nlive = false;
        if (more) lf_fetch_stream<N, T>(A, L, it + n_tensor, ns, ne, nlive);
        // the wavefront's entry slots: rows in, x~ and w_n out
        T *slots = s_stage + (size_t)wv * kWave * SLOT;
        T *mine = slots + (size_t)lane * SLOT;
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int k = 0; k < JP; k += 4)
                *(s3_v4f_m *)(mine + n * JP + k) = s3_v4f_m{u[n][k], u[n][k + 1], u[n][k + 2], u[n][k + 3]};
        // a wavefront contracts only its own slots, so it waits only for
        // itself, except before the first tile (staged core, zeroed tables)
        if (first) __syncthreads();
        else wave_lds_sync();
        mfma_contract_wave<N, JP, OP>(slots, s_g);
        wave_lds_sync();
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
        __syncthreads();  // the slots are reused for the hot-row staging below
        T q = T(0), LG = T(0);
        if (live) {
            const uint2 ms = cs.ms;
            q = -(cs.xv - xhat);
            LG = T(1);
#pragma unroll
            for (int n = 0; n < N; ++n) {
                const T reg = cs.reg[n];
                T ww = T(0), uu = T(0);
#pragma unroll
                for (int k = 0; k < JP; ++k) {
                    ww = fmaT(w[n][k], w[n][k], ww);
                    uu = fmaT(u[n][k], u[n][k], uu);
                }
                LG *= uu;
                const T ell = ww + reg;
                const int pos = lf_field(ms, n);
                if (pos >= 0) {
                    T *t = s_stage + (size_t)n * W * kTile + pos;
#pragma unroll
                    for (int k = 0; k < JP; ++k) t[k * kTile] = fmaT(q, w[n][k], reg * u[n][k]);
                    t[JP * kTile] = ell;
                } else {
                    const T d = kappa * eta * ell;
                    const T step = eta / (d > T(1) ? d : T(1));
                    T *r = A.U[n] + (int64_t)rows[n] * (EXACT ? JP : A.J[n]);
#pragma unroll
                    for (int k = 0; k < JP; ++k)
                        if (EXACT || k < A.J[n]) r[k] = u[n][k] - step * fmaT(q, w[n][k], reg * u[n][k]);
                }
            }
        }
        {
            const T lg = wave_sum(LG);
            const uint64_t bal = __ballot(live);
            if (lane == 0) {
                s_misc[2 * wv] = lg;
                s_misc[2 * wv + 1] = (T)__popcll(bal);
            }
        }
        __syncthreads();
        lf_chunk_pass<JP, N, T, true>(s_stage, s_tab, L.chunks + (size_t)tile * N * kTile, L.nchunks + tile * N,
                                      L.H);
        __syncthreads();
        if (tid == 0) {
            for (int x = 0; x < NWV; ++x) {
                lg_tot += s_misc[2 * x];
                cnt_tot += s_misc[2 * x + 1];
            }
        }
        if constexpr (N == 4) {
            core_grad_mx4_acc<OP>(q, u, s_stage, cacc);  // ends with a barrier
        } else {
            T *s_q = s_stage;                   // [kTile][JP]  q * u^(1)
            T *s_u = s_q + kTile * JP;          // [kTile][N - 1][JP]
#pragma unroll
            for (int k = 0; k < JP; ++k) s_q[tid * JP + k] = q * u[0][k];
#pragma unroll
            for (int n = 1; n < N; ++n)
#pragma unroll
                for (int k = 0; k < JP; ++k) s_u[((size_t)tid * (N - 1) + (n - 1)) * JP + k] = u[n][k];
            __syncthreads();
            // this workgroup's own core partial: stored by the first tile, added to after
            if constexpr (OP == kOpBF16) core_tile_mfma_bf16<N, JP, kTile>(s_q, s_u, core, kTile, !first);
            else core_tile_mfma<N, JP, kChunk>(s_q, s_u, core, !first);
            __syncthreads();
        }
        first = false;
        if (more) {
            cs = ns;
            e = ne;
            live = nlive;
        }
    }
    if constexpr (N == 4) core_grad_mx4_store(cacc, core);
    if (tid == 0) {
        core[KP] = lg_tot;
        core[KP + 1] = cnt_tot;
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
    int64_t KP;                             // padded core size JP^N (JP: hyper-diagonal)
    int cp;                                 // hyper-diagonal core
    void *mx_img;                           // matrix-core operand image of the core, kept current
    int mx_kind;                            // 0: none; 1/2: 4-way BF16/FP32; 3/4: 3-way BF16/FP32
};

constexpr int kApplyThreads = 256;
constexpr int kXcds = 8;  // workgroups are dealt to the XCDs round robin

// blocks [0, groups * H): one hot row each; blocks after: 16 core elements
// each (in the zero-padded JP^N layout).  Neighbouring hot rows and core
// chunks share cache lines of the partials, so the launch index is mapped
// to give each XCD (and its L2) one contiguous range of them.
S3_DEV int64_t lf_xcd_block(int64_t b, int64_t per_xcd) { return (b % kXcds) * per_xcd + b / kXcds; }

template <int N, typename T>
__global__ __launch_bounds__(kApplyThreads) void k_lf_apply(LFApplyArgs a, int H, int JP, T *__restrict__ G,
                                                            T *__restrict__ Gp, int J0, int J1, int J2, int J3,
                                                            T reg_core, T eta, T kappa, int64_t n_blocks) {
    constexpr int NW = kApplyThreads / kWave;
    const int64_t blk = lf_xcd_block(blockIdx.x, gridDim.x / kXcds);
    if (blk >= n_blocks) return;
    __shared__ T s_red[32 * NW];
    const int tid = threadIdx.x;
    const int nrowblk = a.groups * H;
    if (blk < nrowblk) {
        const int g = (int)(blk / H), slot = (int)(blk % H);
        const int row = a.hot_row[g][slot];
        if (row < 0) return;  // uniform over the block
        // lane groups of KW lanes read one workgroup's JP + 1 contiguous
        // values each (lane k: element k); NS groups stride over workgroups
        const int W = JP + 1;
        const int lk = (W <= 16) ? 4 : 5, KW = 1 << lk, NS = kApplyThreads >> lk;
        const int k = tid & (KW - 1), sub = tid >> lk;
        // eight loads in flight per lane, eight running sums
        constexpr int UN = 8;
        T acc8[UN];
#pragma unroll
        for (int i = 0; i < UN; ++i) acc8[i] = T(0);
        auto sweep = [&](const T *src, size_t stride, int64_t nwg) {
            int64_t b = sub;
            for (; b + (UN - 1) * NS < nwg; b += UN * NS) {
                T v[UN];
#pragma unroll
                for (int i = 0; i < UN; ++i) v[i] = src[(b + i * NS) * stride + k];
#pragma unroll
                for (int i = 0; i < UN; ++i) acc8[i] += v[i];
            }
            for (int i = 0; b < nwg; b += NS, ++i) acc8[i & (UN - 1)] += src[b * stride + k];
        };
        if (k < W) {
            if (g < N) sweep((const T *)a.tab_t + ((size_t)g * H + slot) * W, (size_t)N * H * W, a.nwg_t);
            for (int m = 0; m < a.M; ++m) {
                int side = -1;
                if (g < N && a.mat_mode[m] == g) side = 0;
                if (g == N + m) side = 1;
                if (side >= 0)
                    sweep((const T *)a.tab_m[m] + ((size_t)side * H + slot) * W, (size_t)2 * H * W, a.nwg_m[m]);
            }
        }
        T acc = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
        // lanes of one wavefront holding the same element
        for (int off = KW; off < kWave; off <<= 1) acc += __shfl_xor(acc, off, kWave);
        const int lane = tid & (kWave - 1), wv = tid / kWave;
        if (lane < KW) s_red[wv * 32 + lane] = acc;
        __syncthreads();
        if (tid >= a.J[g]) return;
        T gk = T(0), Lsum = T(0);
#pragma unroll 4
        for (int w = 0; w < NW; ++w) {
            gk += s_red[w * 32 + tid];
            Lsum += s_red[w * 32 + JP];
        }
        if (Lsum != T(0)) {
            const T d = kappa * eta * Lsum;
            const T step = eta / (d > T(1) ? d : T(1));
            T *p = (T *)a.P[g] + (int64_t)row * a.J[g];
            p[tid] -= step * gk;
        }
        return;
    }
    // core: lane el of phase ph sums element el of this block over the
    // workgroups ph, ph + PH, ...; the phases are then added in order.  Every
    // lane also sums the two trailing entries (core curvature, entry count).
    constexpr int PH = kApplyThreads / 16;
    __shared__ T s_part[3][PH][17];
    const int el = tid & 15, ph = tid >> 4;
    const int64_t cs = a.KP + 2;
    const int64_t jp = (blk - nrowblk) * 16 + el;
    const T *ct = (const T *)a.core_t;
    T e4[4] = {T(0), T(0), T(0), T(0)}, l4[4] = {T(0), T(0), T(0), T(0)}, c4[4] = {T(0), T(0), T(0), T(0)};
    const int64_t jr = jp < a.KP ? jp : a.KP;  // lanes past the end re-read a valid column
    int64_t b = ph;
    for (; b + 3 * PH < a.nwg_t; b += 4 * PH) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T *row = ct + (b + PH * i) * cs;
            e4[i] += row[jr];
            l4[i] += row[a.KP];
            c4[i] += row[a.KP + 1];
        }
    }
    for (; b < a.nwg_t; b += PH) {
        const T *row = ct + b * cs;
        e4[0] += row[jr];
        l4[0] += row[a.KP];
        c4[0] += row[a.KP + 1];
    }
    s_part[0][ph][el] = (e4[0] + e4[1]) + (e4[2] + e4[3]);
    s_part[1][ph][el] = (l4[0] + l4[1]) + (l4[2] + l4[3]);
    s_part[2][ph][el] = (c4[0] + c4[1]) + (c4[2] + c4[3]);
    __syncthreads();
    if (ph != 0 || jp >= a.KP) return;
    T gsum = T(0), LG = T(0), cnt = T(0);
#pragma unroll 4
    for (int q = 0; q < PH; ++q) {
        gsum += s_part[0][q][el];
        LG += s_part[1][q][el];
        cnt += s_part[2][q][el];
    }
    if (cnt == T(0)) return;
    // padded index -> core index (skip the zero padding)
    const int Js[4] = {J0, J1, J2, J3};
    int64_t rem = jp, j = 0, mul = 1;
    for (int n = (a.cp ? 0 : N - 1); n >= 0; --n) {
        const int jn = (int)(rem % JP);
        rem /= JP;
        if (jn >= Js[n]) return;
        j += jn * mul;
        mul *= Js[n];
    }
    const T Lsum = LG + cnt * reg_core;
    const T d = kappa * eta * Lsum;
    const T step = eta / (d > T(1) ? d : T(1));
    const T gnew = G[j] - step * (gsum + cnt * reg_core * G[j]);
    G[j] = gnew;
    Gp[jp] = gnew;
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (N == 4) {
            if (a.mx_kind == 1) mfma_image_write<4, 8, kOpBF16>(a.mx_img, (int)jp, gnew);
            else if (a.mx_kind == 2) mfma_image_write<4, 8, kOpF32>(a.mx_img, (int)jp, gnew);
        } else {
            if (a.mx_kind == 3) mfma_image_write<3, 16, kOpBF16>(a.mx_img, (int)jp, gnew);
            else if (a.mx_kind == 4) mfma_image_write<3, 16, kOpF32>(a.mx_img, (int)jp, gnew);
        }
    }
}

// ---------------------------------------------------------------- metadata

// Per-entry stream built once at bind time, read coalesced by the round
// kernels instead of three random count/slot lookups per entry and mode.
struct LFMetaSrc {
    const int32_t *hot_slot[kMaxN + kMaxM];
    const int32_t *cnt[kMaxN];
};

template <typename T>
__global__ void k_lf_meta_tensor(const int32_t *__restrict__ idx, int64_t nnz, int N, LFMetaSrc src, T lambda_reg,
                                  uint2 *__restrict__ slot_out, T *__restrict__ reg_out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h[2] = {0xffffffffu, 0xffffffffu};
        for (int n = 0; n < N; ++n) {
            const int32_t row = idx[(int64_t)n * nnz + e];
            const uint32_t sl = (uint32_t)(uint16_t)(int16_t)src.hot_slot[n][row];
            h[n >> 1] = (n & 1) ? ((h[n >> 1] & 0xffffu) | (sl << 16)) : ((h[n >> 1] & 0xffff0000u) | sl);
            reg_out[(int64_t)n * nnz + e] = lambda_reg / (T)src.cnt[n][row];
        }
        slot_out[e] = make_uint2(h[0], h[1]);
    }
}

template <typename T>
__global__ void k_lf_meta_matrix(const int32_t *__restrict__ row, const int32_t *__restrict__ col, int64_t nnz,
                                 const int32_t *__restrict__ slot_u, const int32_t *__restrict__ slot_v,
                                 const int32_t *__restrict__ cntV, T lm_lreg, uint32_t *__restrict__ slot_out,
                                 T *__restrict__ rv_out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t su = (uint32_t)(uint16_t)(int16_t)slot_u[row[e]];
        const uint32_t sv = (uint32_t)(uint16_t)(int16_t)slot_v[col[e]];
        slot_out[e] = su | (sv << 16);
        rv_out[e] = lm_lreg / (T)cntV[col[e]];
    }
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
    void *tab_t = nullptr, *core_t = nullptr;
    uint2 *meta_slot = nullptr;
    uint32_t *t_chunks = nullptr;
    int32_t *t_nchunks = nullptr;
    uint32_t *m_chunks[kMaxM] = {};
    int32_t *m_nchunks[kMaxM] = {};
    void *meta_reg = nullptr;
    uint32_t *meta_mslot[kMaxM] = {};
    void *meta_rv[kMaxM] = {};
    void *tab_m[kMaxM] = {};
    uint64_t seed = 0;
    bool ready = false;
    // per-launch state for the tensor kernel (set by lockfree_epoch)
    uint64_t pa = 1, pb = 0;
    LFApplyArgs apply{};
    const int32_t *cntV[kMaxM] = {};
    s3_buffers b{};
    // this round's matrix tiles (set by lockfree_epoch before the launch)
    int64_t m_base[kMaxM] = {}, m_count[kMaxM] = {};
    uint64_t mpa[kMaxM] = {}, mpb[kMaxM] = {};
    int mat_mode[kMaxM] = {};
    int mat_J[kMaxM] = {};
    double lambda_m = 0.0;
};

constexpr size_t kLfLdsBudget = 64 * 1024;

// hot rows per group: the requested count (power of two, <= 256) or, for 0,
// the largest that lets the tensor kernel's LDS fit the budget (0: none
// fits).  A negative request keeps a minimal table but marks no row hot.
inline int lf_hot_rows(int N, int JP, size_t tsize, int requested) {
    const size_t staging = (std::max((size_t)kTile * N * (JP + 1), (size_t)kTile * N * JP) + 2 * (kTile / kWave)) * tsize;
    for (int H = 256; H >= 16; H /= 2)
        if ((requested <= 0 || H <= requested) && staging + (size_t)N * H * (JP + 1) * tsize <= kLfLdsBudget)
            return requested < 0 ? std::min(H, 16) : H;
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
    s.meta_slot = c.template take<uint2>((size_t)x_nnz);
    s.meta_reg = c.template take<T>((size_t)x_nnz * N);
    s.t_chunks = c.template take<uint32_t>((size_t)tt * N * kTile);
    s.t_nchunks = c.template take<int32_t>((size_t)tt * N);
    for (int m = 0; m < M; ++m) {
        s.meta_mslot[m] = c.template take<uint32_t>((size_t)std::max<int64_t>(y_nnz[m], 1));
        s.meta_rv[m] = c.template take<T>((size_t)std::max<int64_t>(y_nnz[m], 1));
        const int64_t mt = (y_nnz[m] + kTile - 1) / kTile;
        s.m_chunks[m] = c.template take<uint32_t>((size_t)mt * 2 * kTile);
        s.m_nchunks[m] = c.template take<int32_t>((size_t)mt * 2);
    }
    s.core_t = c.template take<T>((size_t)s.max_t_wg * (KP + 2));
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
    s.lambda_m = d.lambda_m;
    for (int m = 0; m < M; ++m) {
        s.mat_mode[m] = d.mat_mode[m];
        s.mat_J[m] = d.rank[d.mat_mode[m]];
    }
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
        const int64_t take = d.hot_rows < 0 ? 0 : std::min<int64_t>(s.H, R);
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
    s.apply.KP = s.KP;
    s.apply.cp = d.core_kind == S3_CORE_CP;
    // per-entry metadata streams
    LFMetaSrc src{};
    for (int g = 0; g < N + M; ++g) src.hot_slot[g] = s.hot_slot[g];
    for (int n = 0; n < N; ++n) src.cnt[n] = cnt[n];
    hipLaunchKernelGGL(k_lf_meta_tensor<T>, dim3(4096), dim3(256), 0, st, buf->x_idx, nX, N, src, (T)d.lambda_reg,
                       s.meta_slot, (T *)s.meta_reg);
    for (int m = 0; m < M; ++m)
        if (y_nnz[m] > 0)
            hipLaunchKernelGGL(k_lf_meta_matrix<T>, dim3(4096), dim3(256), 0, st, buf->y_row[m], buf->y_col[m],
                               y_nnz[m], s.hot_slot[d.mat_mode[m]], s.hot_slot[N + m], cntV[m],
                               (T)(d.lambda_m * d.lambda_reg), s.meta_mslot[m], (T *)s.meta_rv[m]);
    // sorted hot positions and chunk descriptors per tile
    if (s.t_tiles > 0) {
        auto ck = (N == 3) ? k_lf_chunks<uint2, 3> : k_lf_chunks<uint2, 4>;
        hipLaunchKernelGGL(ck, dim3((unsigned)s.t_tiles), dim3(kTile), 0, st, s.meta_slot, nX, s.t_chunks,
                           s.t_nchunks);
    }
    for (int m = 0; m < M; ++m)
        if (s.m_tiles[m] > 0)
            hipLaunchKernelGGL((k_lf_chunks<uint32_t, 2>), dim3((unsigned)s.m_tiles[m]), dim3(kTile), 0, st,
                               s.meta_mslot[m], y_nnz[m], s.m_chunks[m], s.m_nchunks[m]);
    if (hipGetLastError() != hipSuccess) {
        err = "building the lock-free chunk tables failed";
        return S3_ERR_HIP;
    }
    s.ready = true;
    return S3_OK;
}

template <typename T> LFArgs<T> lf_args(const LockFreeState &s, int64_t n_tiles, int64_t base, T *tab, T *core) {
    LFArgs<T> L{};
    for (int g = 0; g < s.N + s.M; ++g) L.hot_slot[g] = s.hot_slot[g];
    L.tab_out = tab;
    L.core_out = core;
    L.meta_slot = s.meta_slot;
    L.chunks = s.t_chunks;
    L.nchunks = s.t_nchunks;
    L.meta_reg = (const T *)s.meta_reg;
    L.H = s.H;
    L.JP = s.JP;
    L.n_tiles = n_tiles;
    L.tile_base = base;
    L.pa = s.pa;
    L.pb = s.pb;
    return L;
}

// Returns the number of tensor workgroups launched (the round's partial tables).
template <int N, int JP, typename T, bool EXACT, int CT = kReuse>
int64_t lockfree_tensor_launch(LockFreeState &s, const TensorArgs<T> &A, const T *Gp, int64_t first, int64_t count,
                               T eta, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                               const void *g_fmt = nullptr) {
    LFArgs<T> L = lf_args<T>(s, s.t_tiles, first, (T *)s.tab_t, (T *)s.core_t);
    LFMatArgs<T> Y{};
    Y.M = s.M;
    Y.lambda_m = (T)s.lambda_m;
    int64_t blocks = count;
    for (int m = 0; m < s.M; ++m) {
        Y.row[m] = s.b.y_row[m];
        Y.col[m] = s.b.y_col[m];
        Y.val[m] = (const T *)s.b.y_val[m];
        Y.nnz[m] = s.y_nnz[m];
        Y.Uc[m] = (T *)s.b.U[s.mat_mode[m]];
        Y.V[m] = (T *)s.b.V[m];
        Y.J[m] = s.mat_J[m];
        Y.cntV[m] = s.cntV[m];
        Y.n_tiles[m] = s.m_tiles[m];
        Y.tile_base[m] = s.m_base[m];
        Y.n_blocks[m] = s.m_count[m];
        Y.pa[m] = s.mpa[m];
        Y.pb[m] = s.mpb[m];
        Y.tab_out[m] = (T *)s.tab_m[m];
        Y.meta_slot[m] = s.meta_mslot[m];
        Y.chunks[m] = s.m_chunks[m];
        Y.nchunks[m] = s.m_nchunks[m];
        Y.meta_rv[m] = (const T *)s.meta_rv[m];
        Y.gu[m] = s.mat_mode[m];
        Y.gv[m] = N + m;
        blocks += s.m_count[m];
    }
    if (blocks <= 0) return count;
    const size_t W = (size_t)JP + 1;
    if constexpr (is_mx(CT)) {
        if constexpr (mfma_shape<N, JP>() && std::is_same<T, float>::value) {
            // tensor workgroups: as many tiles each as two resident workgroups
            // per CU need to cover the round, spread evenly
            const int64_t per = std::max<int64_t>(1, (count + kMxResident - 1) / kMxResident);
            const int64_t nwg = (count + per - 1) / per;
            blocks = blocks - count + nwg;
            constexpr int OP = (CT == kMfma16) ? kOpBF16 : kOpF32;
            // staged core, tables and misc (padded to 16 bytes), then the larger
            // of the entry slots and the hot-row staging
            const size_t stage = std::max((size_t)kTile * MfmaDims<N, JP>::SLOT, (size_t)N * kTile * W);
            const size_t main = mfma_core_bytes<N, JP, OP>() +
                                ((size_t)N * s.H * W + 4 * ((2 * (kTile / kWave) + 3) / 4) + stage) * sizeof(T);
            const size_t smem = std::max(main, (size_t)2 * (s.H * W + kTile * W) * sizeof(T));
            static bool attr = false;  // per instantiation: allow more than 64 KiB of dynamic LDS
            if (!attr) {
                (void)hipFuncSetAttribute((const void *)k_lf_tensor_mx<N, JP, EXACT, CT>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
                attr = true;
            }
            hipExtLaunchKernelGGL((k_lf_tensor_mx<N, JP, EXACT, CT>), dim3((unsigned)blocks), dim3(kTile),
                                  (uint32_t)smem, st, e0, e1, 0, A, g_fmt, L, Y, nwg, count, eta, (T)(N + 1));
            return nwg;
        }
        return count;
    }
    const size_t smem = std::max((size_t)N * (s.H * W + kTile * W) + 2 * (kTile / kWave),
                                 (size_t)2 * (s.H * W + kTile * W)) * sizeof(T);
    // e0/e1 (profiling, may be null) take the dispatch's own start and end
    hipExtLaunchKernelGGL((k_lf_tensor<N, JP, T, EXACT, CT>), dim3((unsigned)blocks), dim3(kTile), (uint32_t)smem, st,
                          e0, e1, 0, A, Gp, L, Y, count, eta, (T)(N + 1));
    return count;
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
    for (int64_t r = 0; r < R; ++r) {
        const int64_t t0 = s.t_tiles * r / R, t1 = s.t_tiles * (r + 1) / R;
        s.pa = tpa;
        s.pb = tpb;
        s.apply.nwg_t = t1 - t0;
        for (int m = 0; m < M; ++m) {
            const int64_t m0 = s.m_tiles[m] * r / R, m1 = s.m_tiles[m] * (r + 1) / R;
            s.m_base[m] = m0;
            s.m_count[m] = std::max<int64_t>(0, m1 - m0);
            s.mpa[m] = mpa[m];
            s.mpb[m] = mpb[m];
            s.apply.nwg_m[m] = s.m_count[m];
        }
        s.apply.nwg_t = tensor_round(t0, t1 - t0, eta, st);  // tensor and matrix tiles, one launch
        const int64_t blocks = (int64_t)(N + M) * s.H + (s.KP + 15) / 16;
        const int64_t grid = (blocks + kXcds - 1) / kXcds * kXcds;
        auto kern = (N == 3) ? k_lf_apply<3, T> : k_lf_apply<4, T>;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kApplyThreads), 0, st, s.apply, s.H, s.JP,
                           (T *)s.b.G, Gp, J[0], J[1], J[2], N > 3 ? J[3] : 1, reg_core, (T)eta, kappa, blocks);
    }
    return S3_OK;
}

}  // namespace s3
