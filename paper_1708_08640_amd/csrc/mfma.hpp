// Dense part of the per-entry contraction on the matrix cores.
//
// A wavefront contracts 64 entries (one per lane) whose factor rows are
// staged in LDS, 32 at a time.  The dense products are (rows x depth) .
// (depth x 32 entries) products on the matrix cores: the core, matricised,
// is the A operand (staged in LDS in the instruction's lane order), and the
// 32 entries' B columns are built in registers.  An output column (one
// entry) lands in lanes j and j + 32, each with half of the rows; the rest
// runs on the VALU in those two lanes, and the values a lane half lacks are
// added with the partner lane (lane ^ 32).
//
// 4-way, rank 8: the core matricised as M[(j1 j2)][(j3 j4)] (64 x 64).  Two
// products of depth 64 whose B columns are the Khatri-Rao products of the
// entry's rows (Definition 1):
//   S_e = M^T (u^(1) o u^(2))_e   (G x_1 u^(1) x_2 u^(2), over j3, j4)
//   R_e = M   (u^(3) o u^(4))_e   (G x_3 u^(3) x_4 u^(4), over j1, j2)
// and from them, with the division-free reuse of Algorithm 3,
//   w_3 = S u^(4), w_4 = S^T u^(3), x~ = w_4 . u^(4),
//   w_1 = R u^(2), w_2 = R^T u^(1).
// Cost per entry: 2 J^N multiply-adds on the matrix cores, and on the VALU
// the 2 J^2 Khatri-Rao products and 4 J^2 multiply-adds.
//
// 3-way, rank 16: the two mode products T1_e = G x_1 u^(1)_e and
// TN_e = G x_3 u^(3)_e (tail 256, depth 16: eight 32-row tiles each); from
// T1: x~, w_2 and w_3, from TN: w_1.  The tail order of each lane half is
// chosen so that w_1 and w_2 are complete inside a lane.  Cost per entry:
// 2 J^N multiply-adds on the matrix cores, about 3 J^(N-1) on the VALU.
//
// Operands: OP = kOpF32 uses v_mfma_f32_32x32x2f32 (FP32 inputs and sums);
// OP = kOpBF16 uses v_mfma_f32_32x32x8bf16_1k (inputs rounded to BF16, round
// to nearest even, FP32 sums).
//
// Lane layouts (checked on gfx950): 32x32x2f32: A[i][k] in lane i + 32 k,
// B[k][j] in lane j + 32 k; 32x32x8bf16_1k: A[i][k] in lane i + 32 (k / 4),
// slot k % 4 (B alike); output D[i][j] in lane j + 32 ((i / 4) % 2),
// register 4 (i / 8) + i % 4.
#pragma once
#include "common.hpp"

namespace s3 {

constexpr int kOpF32 = 0;
constexpr int kOpBF16 = 1;

typedef float s3_v16f __attribute__((ext_vector_type(16)));
typedef float s3_v4f_m __attribute__((ext_vector_type(4)));
typedef short s3_v4s __attribute__((ext_vector_type(4)));

template <int N, int JP> constexpr bool mfma_shape() { return (N == 4 && JP == 8) || (N == 3 && JP == 16); }

template <int N, int JP> struct MfmaDims {
    static constexpr int TL = JP * JP;                  // output rows of one product (64 or 256)
    static constexpr int NQ = TL / 32;                  // 32-row tiles
    static constexpr int KD = (N == 4) ? JP * JP : JP;  // depth of one product (64 or 16)
    static constexpr int SLOT = N * JP + 4;             // floats per entry slot in LDS
};

template <int OP, int KD> struct MfmaOp {
    static constexpr int NC = (OP == kOpBF16) ? KD / 8 : KD / 2;  // instructions per tile (K chunks)
    static constexpr int V = (OP == kOpBF16) ? 4 : 1;             // operand values per lane per chunk
};

// values and bytes of the staged core operands (both products)
template <int N, int JP, int OP> constexpr int mfma_core_count() {
    using O = MfmaOp<OP, MfmaDims<N, JP>::KD>;
    return 2 * MfmaDims<N, JP>::NQ * kWave * O::NC * O::V;
}
template <int N, int JP, int OP> constexpr int mfma_core_bytes() {
    return mfma_core_count<N, JP, OP>() * (OP == kOpBF16 ? 2 : 4);
}

// Place of operand element (lane, chunk c, value v) of tile q of product prod
// in the staged image.  A lane's values come in 16-byte groups, and group g
// of all 64 lanes is stored contiguously, so that a wavefront's wide LDS reads
// of one group touch consecutive bank quads.
template <int N, int JP, int OP> S3_DEV int mfma_img_index(int prod, int q, int lane, int c, int v) {
    using D = MfmaDims<N, JP>;
    using O = MfmaOp<OP, D::KD>;
    constexpr int E = O::NC * O::V;              // values per lane
    constexpr int GV = (OP == kOpBF16) ? 8 : 4;  // values per 16-byte group
    const int e = c * O::V + v;
    return (prod * D::NQ + q) * kWave * E + ((e / GV) * kWave + lane) * GV + e % GV;
}

// Two FP32 values to a BF16 pair (round to nearest even; one
// v_cvt_pk_bf16_f32), low half first
typedef __bf16 s3_bf2 __attribute__((ext_vector_type(2)));
S3_DEV uint32_t bf16x2(float lo, float hi) {
    const s3_bf2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}
S3_DEV s3_v4s bf16x4(float a, float b, float c, float d) {
    const uint32_t lo = bf16x2(a, b), hi = bf16x2(c, d);
    return s3_v4s{(short)(lo & 0xffffu), (short)(lo >> 16), (short)(hi & 0xffffu), (short)(hi >> 16)};
}

// 3-way: tail position held by output register r of tile q in lane half h,
// with (x, y) the tail's mode indices (modes 2, 3 for T1, 1, 2 for TN):
// x = 8 h + q, y = r, so half h owns x in [8h, 8h + 8).
S3_DEV int mfma_tail3(int q, int h, int r) { return (8 * h + q) * 16 + r; }

// Stage the core operands of both products (all threads of the grid; Gp is
// the zero-padded JP^N core, row-major), each value at mfma_img_index of its
// (product, tile, lane, chunk, value).  Output row i of tile q is row 32 q + i
// of the product; depth index k.
//   4-way: product 0 is M^T (row (j3 j4), depth (j1 j2)), product 1 is M;
//   3-way: product 0 is T1 (row = tail (j2 j3), depth j1), product 1 is TN
//          (row = tail (j1 j2), depth j3).
template <int N, int JP, int OP>
S3_DEV void mfma_stage_core(const float *__restrict__ Gp, void *__restrict__ s_g) {
    using D = MfmaDims<N, JP>;
    using O = MfmaOp<OP, D::KD>;
    constexpr int total = mfma_core_count<N, JP, OP>();
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < total; x += gridDim.x * blockDim.x) {
        const int v = x % O::V;
        int t = x / O::V;
        const int c = t % O::NC;
        t /= O::NC;
        const int lane = t % kWave;
        t /= kWave;
        const int q = t % D::NQ, prod = t / D::NQ;
        const int i = lane & 31, kh = lane >> 5;
        const int k = (OP == kOpBF16) ? 8 * c + 4 * kh + v : 2 * c + kh;
        float g;
        if constexpr (N == 4) {
            const int row = 32 * q + i;
            g = (prod == 0) ? Gp[k * 64 + row] : Gp[row * 64 + k];
        } else {
            const int h = (i >> 2) & 1, r = 4 * (i >> 3) + (i & 3);
            const int tail = mfma_tail3(q, h, r);
            g = (prod == 0) ? Gp[k * D::TL + tail] : Gp[tail * JP + k];
        }
        const int y = mfma_img_index<N, JP, OP>(prod, q, lane, c, v);
        if constexpr (OP == kOpBF16) ((unsigned short *)s_g)[y] = (unsigned short)(bf16x2(g, 0.f) & 0xffffu);
        else ((float *)s_g)[y] = g;
    }
}

// The operand layout above written once per core value, one element per
// thread (the round and batch kernels then copy it into LDS with wide loads).
template <int N, int JP, int OP>
__global__ __launch_bounds__(256) void k_mx_format(const float *__restrict__ Gp, void *__restrict__ out) {
    mfma_stage_core<N, JP, OP>(Gp, out);
}

// One core value written into the operand image, at both of its places:
// the inverse of mfma_stage_core's mapping, for a kernel that updates the
// core element by element (jp: index in the zero-padded JP^N core).
template <int N, int JP, int OP> S3_DEV void mfma_image_write(void *img, int jp, float g) {
    using D = MfmaDims<N, JP>;
    using O = MfmaOp<OP, D::KD>;
#pragma unroll
    for (int prod = 0; prod < 2; ++prod) {
        int row, k;
        if constexpr (N == 4) {
            row = prod == 0 ? (jp & 63) : (jp >> 6);
            k = prod == 0 ? (jp >> 6) : (jp & 63);
        } else {
            row = prod == 0 ? jp % D::TL : jp / JP;  // the tail
            k = prod == 0 ? jp / D::TL : jp % JP;
        }
        int q, i;
        if constexpr (N == 4) {
            q = row >> 5;
            i = row & 31;
        } else {
            const int x = row >> 4, r = row & 15, h = x >> 3;
            q = x & 7;
            i = 8 * (r >> 2) + 4 * h + (r & 3);
        }
        const int c = (OP == kOpBF16) ? k >> 3 : k >> 1;
        const int kh = (OP == kOpBF16) ? (k >> 2) & 1 : k & 1;
        const int v = (OP == kOpBF16) ? k & 3 : 0;
        const int x = mfma_img_index<N, JP, OP>(prod, q, i + 32 * kh, c, v);
        if constexpr (OP == kOpBF16) ((unsigned short *)img)[x] = (unsigned short)(bf16x2(g, 0.f) & 0xffffu);
        else ((float *)img)[x] = g;
    }
}

// Copy the formatted operands into LDS (all threads of the block)
template <int N, int JP, int OP> S3_DEV void mfma_load_core(const void *__restrict__ g, void *__restrict__ s_g) {
    constexpr int n16 = mfma_core_bytes<N, JP, OP>() / 16;
    const uint4 *src = (const uint4 *)g;
    uint4 *dst = (uint4 *)s_g;
#pragma unroll
    for (int i = 0; i < (n16 + 255) / 256; ++i) {
        const int x = i * 256 + threadIdx.x;
        if (x < n16) dst[x] = src[x];
    }
}

// B operand chunks of one entry column (the lane half kh takes its K values)
template <int OP, int KD> struct MfmaB {
    typename std::conditional<OP == kOpBF16, s3_v4s, float>::type c[MfmaOp<OP, KD>::NC];
};

// 3-way: the column is one of the entry's rows
template <int OP, int JP> S3_DEV MfmaB<OP, JP> mfma_b_of(const float *row, int kh) {
    MfmaB<OP, JP> b;
#pragma unroll
    for (int c = 0; c < MfmaOp<OP, JP>::NC; ++c) {
        if constexpr (OP == kOpBF16) {
            const float *r = row + 8 * c + 4 * kh;
            b.c[c] = bf16x4(r[0], r[1], r[2], r[3]);
        } else {
            b.c[c] = row[2 * c + kh];
        }
    }
    return b;
}

// 4-way: the column is the Khatri-Rao product (a o b)[8 x + y] = a[x] b[y] of
// two rows of 8, formed in FP32 (then rounded once for BF16 operands)
template <int OP> S3_DEV MfmaB<OP, 64> mfma_b_kr(const float (&a)[8], const float (&b)[8], int kh) {
    MfmaB<OP, 64> o;
    if constexpr (OP == kOpBF16) {
        float bh[4];  // depth 8 c + 4 kh + v: x = c, y = 4 kh + v
#pragma unroll
        for (int v = 0; v < 4; ++v) bh[v] = kh ? b[4 + v] : b[v];
#pragma unroll
        for (int c = 0; c < 8; ++c) o.c[c] = bf16x4(a[c] * bh[0], a[c] * bh[1], a[c] * bh[2], a[c] * bh[3]);
    } else {
        float bh[4];  // depth 2 c + kh: x = c / 4, y = 2 (c % 4) + kh
#pragma unroll
        for (int r = 0; r < 4; ++r) bh[r] = kh ? b[2 * r + 1] : b[2 * r];
#pragma unroll
        for (int c = 0; c < 32; ++c) o.c[c] = a[c >> 2] * bh[c & 3];
    }
    return o;
}

// One 32 x 32 output tile: product prod, tile q
template <int N, int JP, int OP>
S3_DEV s3_v16f mfma_tile(const void *s_g, int prod, int q, int lane, const MfmaB<OP, MfmaDims<N, JP>::KD> &b) {
    using D = MfmaDims<N, JP>;
    using O = MfmaOp<OP, D::KD>;
    s3_v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // the lane's 16-byte groups (mfma_img_index): two chunks each for BF16,
    // four for FP32
    if constexpr (OP == kOpBF16) {
        const unsigned short *a = (const unsigned short *)s_g + mfma_img_index<N, JP, OP>(prod, q, lane, 0, 0);
#pragma unroll
        for (int c = 0; c < O::NC; ++c) {
            const s3_v4s av = *(const s3_v4s *)(a + (c >> 1) * kWave * 8 + (c & 1) * 4);
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, b.c[c], acc, 0, 0, 0);
        }
    } else {
        const float *a = (const float *)s_g + mfma_img_index<N, JP, OP>(prod, q, lane, 0, 0);
        float av[O::NC];
#pragma unroll
        for (int c = 0; c < O::NC; c += 4) {
            const s3_v4f_m t = *(const s3_v4f_m *)(a + (c >> 2) * kWave * 4);  // 16-byte aligned group
            av[c] = t[0];
            av[c + 1] = t[1];
            av[c + 2] = t[2];
            av[c + 3] = t[3];
        }
#pragma unroll
        for (int c = 0; c < O::NC; ++c) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[c], b.c[c], acc, 0, 0, 0);
    }
    return acc;
}

// Order this wavefront's LDS writes before its later LDS reads (by any of its
// lanes): the wavefront's LDS instructions complete in issue order, so only
// the compiler has to be kept from moving them.
S3_DEV void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The wavefront's 64 entries: slot s (s = 0..63) of `slots` holds entry s's
// rows u^(1) | ... | u^(N) (JP each, zero padded) and receives, in place,
// w_1 | ... | w_N | x~.  Every lane of the wavefront must call it.
template <int N, int JP, int OP>
S3_DEV void mfma_contract_wave(float *slots, const void *s_g) {
    static_assert(mfma_shape<N, JP>(), "matrix-core contraction: N = 4 with JP = 8, or N = 3 with JP = 16");
    using D = MfmaDims<N, JP>;
    const int lane = threadIdx.x & (kWave - 1);
    const int j = lane & 31, h = lane >> 5;
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        float *slot = slots + (32 * pass + j) * D::SLOT;
        if constexpr (N == 4) {
            float a1[8], a2[8], a3[8], a4[8];
#pragma unroll
            for (int k = 0; k < 8; k += 4) {
                const s3_v4f_m x1 = *(const s3_v4f_m *)(slot + k), x2 = *(const s3_v4f_m *)(slot + 8 + k);
                const s3_v4f_m x3 = *(const s3_v4f_m *)(slot + 16 + k), x4 = *(const s3_v4f_m *)(slot + 24 + k);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    a1[k + v] = x1[v];
                    a2[k + v] = x2[v];
                    a3[k + v] = x3[v];
                    a4[k + v] = x4[v];
                }
            }
            const MfmaB<OP, 64> b12 = mfma_b_kr<OP>(a1, a2, h);
            const MfmaB<OP, 64> b34 = mfma_b_kr<OP>(a3, a4, h);
            // S rows (j3 j4) = 32 t + 8 g + 4 h + v: j3 = 4 t + g, j4 = 4 h + v; R rows
            // (j1 j2) likewise: j1 = 4 t + g, j2 = 4 h + v (register 4 g + v of tile t)
            const s3_v16f S0 = mfma_tile<N, JP, OP>(s_g, 0, 0, lane, b12);
            const s3_v16f S1 = mfma_tile<N, JP, OP>(s_g, 0, 1, lane, b12);
            const s3_v16f R0 = mfma_tile<N, JP, OP>(s_g, 1, 0, lane, b34);
            const s3_v16f R1 = mfma_tile<N, JP, OP>(s_g, 1, 1, lane, b34);
            float a2h[4], a4h[4];  // u^(2), u^(4) at this half's indices 4h .. 4h + 3
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                a2h[v] = h ? a2[4 + v] : a2[v];
                a4h[v] = h ? a4[4 + v] : a4[v];
            }
            float w4h[4] = {0.f, 0.f, 0.f, 0.f}, w2h[4] = {0.f, 0.f, 0.f, 0.f};
            float w3p[8], w1p[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) { w3p[k] = 0.f; w1p[k] = 0.f; }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int x = 4 * t + g;
                        const float sv = t ? S1[4 * g + v] : S0[4 * g + v];
                        const float rv = t ? R1[4 * g + v] : R0[4 * g + v];
                        w4h[v] = fmaf(sv, a3[x], w4h[v]);    // w_4[4h + v] = sum_j3 S u^(3)
                        w3p[x] = fmaf(sv, a4h[v], w3p[x]);   // w_3[j3], this half's j4
                        w2h[v] = fmaf(rv, a1[x], w2h[v]);    // w_2[4h + v] = sum_j1 R u^(1)
                        w1p[x] = fmaf(rv, a2h[v], w1p[x]);   // w_1[j1], this half's j2
                    }
            float xp = 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) xp = fmaf(w4h[v], a4h[v], xp);
            const float xt = xp + __shfl_xor(xp, 32, kWave);
            // this lane keeps indices 4h .. 4h + 3 of w_1 and w_3; the partner
            // sends its partial sums at those indices
            float w1o[4], w3o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float s1 = h ? w1p[k] : w1p[4 + k], s3 = h ? w3p[k] : w3p[4 + k];
                const float m1 = h ? w1p[4 + k] : w1p[k], m3 = h ? w3p[4 + k] : w3p[k];
                w1o[k] = m1 + __shfl_xor(s1, 32, kWave);
                w3o[k] = m3 + __shfl_xor(s3, 32, kWave);
            }
            // results in place (the pair's rows are no longer read)
            *(s3_v4f_m *)(slot + 4 * h) = s3_v4f_m{w1o[0], w1o[1], w1o[2], w1o[3]};
            *(s3_v4f_m *)(slot + 8 + 4 * h) = s3_v4f_m{w2h[0], w2h[1], w2h[2], w2h[3]};
            *(s3_v4f_m *)(slot + 16 + 4 * h) = s3_v4f_m{w3o[0], w3o[1], w3o[2], w3o[3]};
            *(s3_v4f_m *)(slot + 24 + 4 * h) = s3_v4f_m{w4h[0], w4h[1], w4h[2], w4h[3]};
            if (h == 0) slot[32] = xt;
        } else {
            const MfmaB<OP, JP> bfirst = mfma_b_of<OP, JP>(slot, h);
            const MfmaB<OP, JP> blast = mfma_b_of<OP, JP>(slot + (N - 1) * JP, h);
            float b[16], c[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                b[k] = slot[16 + k];
                c[k] = slot[32 + k];
            }
            float bh[8];  // u^(2) at this half's indices 8h .. 8h + 7
#pragma unroll
            for (int k = 0; k < 8; ++k) bh[k] = h ? b[8 + k] : b[k];
            float R[8], w1l[8], w3p[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) w3p[k] = 0.f;
            float xp = 0.f;
            s3_v16f t1 = mfma_tile<N, JP, OP>(s_g, 0, 0, lane, bfirst);
            s3_v16f tn = mfma_tile<N, JP, OP>(s_g, 1, 0, lane, blast);
#pragma unroll
            for (int q = 0; q < D::NQ; ++q) {
                s3_v16f t1n = t1, tnn = tn;
                if (q + 1 < D::NQ) {
                    t1n = mfma_tile<N, JP, OP>(s_g, 0, q + 1, lane, bfirst);
                    tnn = mfma_tile<N, JP, OP>(s_g, 1, q + 1, lane, blast);
                }
                // T1 tile: (j2, j3) = (8h + q, r)
                float S = 0.f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    S = fmaf(t1[r], c[r], S);                  // w_2[j2]
                    w3p[r] = fmaf(t1[r], bh[q], w3p[r]);       // w_3[j3] (this half's j2)
                }
                R[q] = S;
                xp = fmaf(S, bh[q], xp);
                // TN tile: (j1, j2) = (8h + q, r)
                float P = 0.f;
#pragma unroll
                for (int r = 0; r < 16; ++r) P = fmaf(tn[r], b[r], P);
                w1l[q] = P;                                    // w_1[j1]
                t1 = t1n;
                tn = tnn;
            }
            const float x = xp + __shfl_xor(xp, 32, kWave);
            float w3o[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float s3 = h ? w3p[k] : w3p[8 + k];
                const float m3 = h ? w3p[8 + k] : w3p[k];
                w3o[k] = m3 + __shfl_xor(s3, 32, kWave);
            }
#pragma unroll
            for (int k = 0; k < 8; k += 4) {
                *(s3_v4f_m *)(slot + 8 * h + k) = s3_v4f_m{w1l[k], w1l[k + 1], w1l[k + 2], w1l[k + 3]};
                *(s3_v4f_m *)(slot + 16 + 8 * h + k) = s3_v4f_m{R[k], R[k + 1], R[k + 2], R[k + 3]};
                *(s3_v4f_m *)(slot + 32 + 8 * h + k) = s3_v4f_m{w3o[k], w3o[k + 1], w3o[k + 2], w3o[k + 3]};
            }
            if (h == 0) slot[48] = x;
        }
    }
}

// Core gradient of the block's 256 entries for a 4-way core with JP = 8:
//   C[j1 j2][j3 j4] = sum_t (q u^(1) o u^(2))_t[j1 j2] (u^(3) o u^(4))_t[j3 j4],
// a (64 x 256) . (256 x 64) product.  Every entry's two 64-value outer
// products are staged in LDS (entry-major rows, padded against bank
// conflicts), a part of the entries at a time; wavefront w computes the 32 x 32
// output tile (w / 2, w % 2).  BF16 operands: v_mfma_f32_32x32x8bf16_1k on
// halves of 128 entries; FP32: v_mfma_f32_32x32x2f32 on quarters of 64.
// Sums in FP32.  `buf` needs 36,864 bytes, 16-byte aligned; core receives
// the 4,096 values (row-major j1 j2 j3 j4, the padded core layout).
// (accumulated into acc, wavefront w's tile; ends with a barrier)
template <int OP>
S3_DEV void core_grad_mx4_acc(float q, const float (&u)[4][8], float *buf, s3_v16f &acc) {
    constexpr int kPart = (OP == kOpBF16) ? 128 : 64;   // entries staged at a time
    constexpr int kRow = (OP == kOpBF16) ? 136 : 132;   // staged row: 128 values + padding
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int rb = wv >> 1, cb = wv & 1, i = lane & 31, kh = lane >> 5;
    float pa[8], pc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        pa[k] = q * u[0][k];
        pc[k] = u[2][k];
    }
#pragma unroll 1
    for (int part = 0; part < 256 / kPart; ++part) {  // the block's 256 entries
        const int tl = tid - part * kPart;
        if (tl >= 0 && tl < kPart) {
            if constexpr (OP == kOpBF16) {
                unsigned short *row = (unsigned short *)buf + (size_t)tl * kRow;
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    uint32_t pw[4], qw[4];
#pragma unroll
                    for (int b = 0; b < 8; b += 2) {
                        pw[b / 2] = bf16x2(pa[a] * u[1][b], pa[a] * u[1][b + 1]);
                        qw[b / 2] = bf16x2(pc[a] * u[3][b], pc[a] * u[3][b + 1]);
                    }
                    *(uint4 *)(row + 8 * a) = make_uint4(pw[0], pw[1], pw[2], pw[3]);
                    *(uint4 *)(row + 64 + 8 * a) = make_uint4(qw[0], qw[1], qw[2], qw[3]);
                }
            } else {
                float *row = buf + (size_t)tl * kRow;
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    *(s3_v4f_m *)(row + 8 * a) = s3_v4f_m{pa[a] * u[1][0], pa[a] * u[1][1], pa[a] * u[1][2], pa[a] * u[1][3]};
                    *(s3_v4f_m *)(row + 8 * a + 4) = s3_v4f_m{pa[a] * u[1][4], pa[a] * u[1][5], pa[a] * u[1][6], pa[a] * u[1][7]};
                    *(s3_v4f_m *)(row + 64 + 8 * a) = s3_v4f_m{pc[a] * u[3][0], pc[a] * u[3][1], pc[a] * u[3][2], pc[a] * u[3][3]};
                    *(s3_v4f_m *)(row + 68 + 8 * a) = s3_v4f_m{pc[a] * u[3][4], pc[a] * u[3][5], pc[a] * u[3][6], pc[a] * u[3][7]};
                }
            }
        }
        __syncthreads();
        if constexpr (OP == kOpBF16) {
            const unsigned short *sb = (const unsigned short *)buf;
#pragma unroll 4
            for (int k0 = 0; k0 < kPart; k0 += 8) {
                s3_v4s a, b;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int t = k0 + 4 * kh + v;
                    a[v] = (short)sb[(size_t)t * kRow + 32 * rb + i];
                    b[v] = (short)sb[(size_t)t * kRow + 64 + 32 * cb + i];
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
            }
        } else {
#pragma unroll 4
            for (int k0 = 0; k0 < kPart; k0 += 2) {
                const int t = k0 + kh;
                const float a = buf[(size_t)t * kRow + 32 * rb + i];
                const float b = buf[(size_t)t * kRow + 64 + 32 * cb + i];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
            }
        }
        __syncthreads();
    }
}

// wavefront w's 32 x 32 tile of the 4-way core gradient, to core (4,096 values)
S3_DEV void core_grad_mx4_store(const s3_v16f &acc, float *__restrict__ core) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int rb = wv >> 1, cb = wv & 1, i = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * kh + (r & 3);
        core[(size_t)(32 * rb + row) * 64 + 32 * cb + i] = acc[r];
    }
}

template <int OP>
S3_DEV void core_grad_mx4(float q, const float (&u)[4][8], float *buf, float *__restrict__ core) {
    s3_v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    core_grad_mx4_acc<OP>(q, u, buf, acc);
    core_grad_mx4_store(acc, core);
}

// Core gradient of a chunk of K entries on the BF16 matrix cores (FP32
// sums): C[j1][tau] = sum_t (q u^(1))_t[j1] (u^(2) o ... o u^(N))_t[tau], as
// (16 x K) x (K x 16 n-tiles) products with v_mfma_f32_16x16x16bf16_1k
// (A[i][k] in lane i + 16 (k / 4), slot k % 4; D[4 (l / 16) + r][l % 16] in
// lane l, register r).  Same operands and output as core_tile_mfma.
template <int N, int JP, int K>
S3_DEV void core_tile_mfma_bf16(const float *s_q, const float *s_u, float *core, int nthreads, bool add = false) {
    constexpr int TAIL = (N == 3) ? JP * JP : JP * JP * JP;
    constexpr int NT = (TAIL + 15) / 16;
    const int NW = nthreads / kWave;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int i16 = lane & 15, kq = lane >> 4;
    for (int nt = wv; nt < NT; nt += NW) {  // uniform over the wave
        const int tau = 16 * nt + i16;
        const bool tv = tau < TAIL;
        int tj[N - 1];
        int r = tv ? tau : 0;
#pragma unroll
        for (int n = N - 2; n >= 0; --n) { tj[n] = r % JP; r /= JP; }
        typedef float v4f __attribute__((ext_vector_type(4)));
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < K; k0 += 16) {
            float av[4], bvv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = k0 + 4 * kq + v;
                av[v] = (i16 < JP) ? s_q[t * JP + i16] : 0.f;
                float bv = s_u[(t * (N - 1)) * JP + tj[0]];
#pragma unroll
                for (int n = 1; n < N - 1; ++n) bv *= s_u[(t * (N - 1) + n) * JP + tj[n]];
                bvv[v] = tv ? bv : 0.f;
            }
            const s3_v4s a = bf16x4(av[0], av[1], av[2], av[3]);
            const s3_v4s b = bf16x4(bvv[0], bvv[1], bvv[2], bvv[3]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        if (tv) {
#pragma unroll
            for (int r2 = 0; r2 < 4; ++r2) {
                const int j1 = 4 * kq + r2;
                if (j1 < JP) {
                    float *c = core + (size_t)j1 * TAIL + tau;
                    *c = add ? *c + acc[r2] : acc[r2];
                }
            }
        }
    }
}

}  // namespace s3
