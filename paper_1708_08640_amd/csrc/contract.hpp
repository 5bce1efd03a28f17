// Per-entry Tucker contractions on one lane.
//
// For one observed entry with factor rows u^(1..N) (held in registers, zero
// padded to JP) and the core G (JP^N, row-major, zero padded), compute in a
// single pass over G:
//   w_n[k] = [G x_{-n} {u}]_k   (the leave-one-out contraction of Eq 8)
//   x~     = G x {u}            (Eq 4)
// Every core element is read once and feeds two fused multiply-adds: one
// into the contraction with the innermost factor (a running partial sum
// that is reused for all outer modes) and one into w_N.  This is the
// paper's reuse of intermediate products (Definition 4, Lemma 2,
// Algorithm 3) in a division-free form: partial contractions are kept and
// re-used instead of dividing the full product by a factor entry.
// Cost: 2 * JP^N FMAs plus O(N * JP^(N-1)).
#pragma once
#include "common.hpp"

namespace s3 {


template <int JP, typename T, typename GP>
S3_DEV void contract3(GP G, const T (&a)[JP], const T (&b)[JP], const T (&c)[JP],
                      T (&w1)[JP], T (&w2)[JP], T (&w3)[JP], T &xhat) {
#pragma unroll
    for (int k = 0; k < JP; ++k) { w2[k] = T(0); w3[k] = T(0); }
#pragma unroll
    for (int j1 = 0; j1 < JP; ++j1) {
        T s1 = T(0);
#pragma unroll
        for (int j2 = 0; j2 < JP; ++j2) {
            const T ab = a[j1] * b[j2];
            T t = T(0);
#pragma unroll
            for (int j3 = 0; j3 < JP; ++j3) {
                const T g = G[(j1 * JP + j2) * JP + j3];
                t = fmaT(g, c[j3], t);          // (G x_3 c)[j1][j2]
                w3[j3] = fmaT(ab, g, w3[j3]);   // (G x_1 a x_2 b)[j3]
            }
            w2[j2] = fmaT(a[j1], t, w2[j2]);
            s1 = fmaT(b[j2], t, s1);
        }
        w1[j1] = s1;
    }
    T x = T(0);
#pragma unroll
    for (int k = 0; k < JP; ++k) x = fmaT(w3[k], c[k], x);
    xhat = x;
}

template <int JP, typename T, typename GP>
S3_DEV void contract4(GP G, const T (&a)[JP], const T (&b)[JP], const T (&c)[JP],
                      const T (&d)[JP], T (&w1)[JP], T (&w2)[JP], T (&w3)[JP], T (&w4)[JP],
                      T &xhat) {
#pragma unroll
    for (int k = 0; k < JP; ++k) { w2[k] = T(0); w3[k] = T(0); w4[k] = T(0); }
#pragma unroll
    for (int j1 = 0; j1 < JP; ++j1) {
        T s1 = T(0);
#pragma unroll
        for (int j2 = 0; j2 < JP; ++j2) {
            const T ab = a[j1] * b[j2];
            T s2 = T(0);
#pragma unroll
            for (int j3 = 0; j3 < JP; ++j3) {
                    const T abc = ab * c[j3];
                T t = T(0);
#pragma unroll
                for (int j4 = 0; j4 < JP; ++j4) {
                    const T g = G[((j1 * JP + j2) * JP + j3) * JP + j4];
                    t = fmaT(g, d[j4], t);
                    w4[j4] = fmaT(abc, g, w4[j4]);
                }
                w3[j3] = fmaT(ab, t, w3[j3]);
                s2 = fmaT(c[j3], t, s2);
            }
            w2[j2] = fmaT(a[j1], s2, w2[j2]);
            s1 = fmaT(b[j2], s2, s1);
        }
        w1[j1] = s1;
    }
    T x = T(0);
#pragma unroll
    for (int k = 0; k < JP; ++k) x = fmaT(w4[k], d[k], x);
    xhat = x;
}

// The single pass above split over S workers by the first core index:
// worker w (uniform over its wavefront) takes j1 = w, w + S, ... -- a[i]
// holds u^(1)[w + S i] and v the other modes' rows -- and returns w_1 at its
// j1, its partial sums of w_2 .. w_N over those j1, and its part of
// x~ = sum_j1 u^(1)[j1] w_1[j1].  The S partials added in a fixed order give
// the single pass's results (up to the order of the additions).
template <int N, int JP, int S, typename T>
S3_DEV void contract_part(const T *__restrict__ G, int w, const T (&a)[(JP + S - 1) / S],
                          const T (&v)[N - 1][JP], T (&w1)[(JP + S - 1) / S], T (&wv)[N - 1][JP],
                          T &xpart) {
    constexpr int NI = (JP + S - 1) / S;
#pragma unroll
    for (int n = 0; n < N - 1; ++n)
#pragma unroll
        for (int k = 0; k < JP; ++k) wv[n][k] = T(0);
    T x = T(0);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        w1[i] = T(0);
        const int j1 = w + S * i;
        if (j1 >= JP) continue;  // uniform
        T s1 = T(0);
        if constexpr (N == 3) {
            const T *Gj = G + j1 * JP * JP;
#pragma unroll
            for (int j2 = 0; j2 < JP; ++j2) {
                const T ab = a[i] * v[0][j2];
                T t = T(0);
#pragma unroll
                for (int j3 = 0; j3 < JP; ++j3) {
                    const T g = Gj[j2 * JP + j3];
                    t = fmaT(g, v[1][j3], t);
                    wv[1][j3] = fmaT(ab, g, wv[1][j3]);
                }
                wv[0][j2] = fmaT(a[i], t, wv[0][j2]);
                s1 = fmaT(v[0][j2], t, s1);
            }
        } else {
            const T *Gj = G + j1 * JP * JP * JP;
#pragma unroll
            for (int j2 = 0; j2 < JP; ++j2) {
                const T ab = a[i] * v[0][j2];
                T s2 = T(0);
#pragma unroll
                for (int j3 = 0; j3 < JP; ++j3) {
                    const T abc = ab * v[1][j3];
                    T t = T(0);
#pragma unroll
                    for (int j4 = 0; j4 < JP; ++j4) {
                        const T g = Gj[(j2 * JP + j3) * JP + j4];
                        t = fmaT(g, v[2][j4], t);
                        wv[2][j4] = fmaT(abc, g, wv[2][j4]);
                    }
                    wv[1][j3] = fmaT(ab, t, wv[1][j3]);
                    s2 = fmaT(v[1][j3], t, s2);
                }
                wv[0][j2] = fmaT(a[i], s2, wv[0][j2]);
                s1 = fmaT(v[0][j2], s2, s1);
            }
        }
        w1[i] = s1;
        x = fmaT(a[i], s1, x);
    }
    xpart = x;
}

// N-generic front end: rows u[n][k], outputs w[n][k]
template <int N, int JP, typename T, typename GP>
S3_DEV void contract(GP G, const T (&u)[N][JP], T (&w)[N][JP], T &xhat) {
    if constexpr (N == 3) {
        contract3<JP, T>(G, u[0], u[1], u[2], w[0], w[1], w[2], xhat);
    } else {
        contract4<JP, T>(G, u[0], u[1], u[2], u[3], w[0], w[1], w[2], w[3], xhat);
    }
}

// Ablation baseline without reuse: x~ and every w_n each take their own
// pass over the core, forming every term from the factor entries afresh
// (the per-entry work of the paper's naive form, Algorithm 2, whose cost
// Lemma 4 compares with the reuse of Algorithm 3).  (N + 1) passes of Jᴺ
// terms with N - 1 products each, against 2 Jᴺ FMAs above.
template <int N, int JP, typename T, typename GP>
S3_DEV void contract_naive(GP G, const T (&u)[N][JP], T (&w)[N][JP], T &xhat) {
    T x = T(0);
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int k = 0; k < JP; ++k) w[n][k] = T(0);
    if constexpr (N == 3) {
#pragma unroll
        for (int j1 = 0; j1 < JP; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < JP; ++j2)
#pragma unroll
                for (int j3 = 0; j3 < JP; ++j3) {
                    const T g = G[(j1 * JP + j2) * JP + j3];
                    x = fmaT(g, u[0][j1] * u[1][j2] * u[2][j3], x);
                    w[0][j1] = fmaT(g, u[1][j2] * u[2][j3], w[0][j1]);
                    w[1][j2] = fmaT(g, u[0][j1] * u[2][j3], w[1][j2]);
                    w[2][j3] = fmaT(g, u[0][j1] * u[1][j2], w[2][j3]);
                }
    } else {
#pragma unroll
        for (int j1 = 0; j1 < JP; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < JP; ++j2)
#pragma unroll
                for (int j3 = 0; j3 < JP; ++j3)
#pragma unroll
                    for (int j4 = 0; j4 < JP; ++j4) {
                        const T g = G[((j1 * JP + j2) * JP + j3) * JP + j4];
                        x = fmaT(g, u[0][j1] * u[1][j2] * u[2][j3] * u[3][j4], x);
                        w[0][j1] = fmaT(g, u[1][j2] * u[2][j3] * u[3][j4], w[0][j1]);
                        w[1][j2] = fmaT(g, u[0][j1] * u[2][j3] * u[3][j4], w[1][j2]);
                        w[2][j3] = fmaT(g, u[0][j1] * u[1][j2] * u[3][j4], w[2][j3]);
                        w[3][j4] = fmaT(g, u[0][j1] * u[1][j2] * u[2][j3], w[3][j4]);
                    }
    }
    xhat = x;
}

// prediction only (Eq 4): same pass without the w_n outputs for outer modes
template <int N, int JP, typename T, typename GP>
S3_DEV T predict(GP G, const T (&u)[N][JP]) {
    T acc = T(0);
    if constexpr (N == 3) {
#pragma unroll
        for (int j1 = 0; j1 < JP; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < JP; ++j2) {
                T t = T(0);
#pragma unroll
                for (int j3 = 0; j3 < JP; ++j3) t = fmaT(G[(j1 * JP + j2) * JP + j3], u[2][j3], t);
                acc = fmaT(u[0][j1] * u[1][j2], t, acc);
            }
    } else {
#pragma unroll
        for (int j1 = 0; j1 < JP; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < JP; ++j2)
#pragma unroll
                for (int j3 = 0; j3 < JP; ++j3) {
                    T t = T(0);
#pragma unroll
                    for (int j4 = 0; j4 < JP; ++j4)
                        t = fmaT(G[((j1 * JP + j2) * JP + j3) * JP + j4], u[3][j4], t);
                    acc = fmaT(u[0][j1] * u[1][j2] * u[2][j3], t, acc);
                }
    }
    return acc;
}

// CP special case (hyper-diagonal core, Section 3's S^3CMTF-CP): g holds
// the JP diagonal values (zero padded), x~ = sum_r g_r prod_n u_n[r] and
// w_n[r] = g_r prod_{m != n} u_m[r]: O(N^2 J) per entry.
template <int N, int JP, typename T, typename GP>
S3_DEV void contract_cp(GP g, const T (&u)[N][JP], T (&w)[N][JP], T &xhat) {
    T x = T(0);
#pragma unroll
    for (int r = 0; r < JP; ++r) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            T p = g[r];
#pragma unroll
            for (int m = 0; m < N; ++m)
                if (m != n) p *= u[m][r];
            w[n][r] = p;
        }
        x = fmaT(w[0][r], u[0][r], x);
    }
    xhat = x;
}

template <int N, int JP, typename T, typename GP> S3_DEV T predict_cp(GP g, const T (&u)[N][JP]) {
    T x = T(0);
#pragma unroll
    for (int r = 0; r < JP; ++r) {
        T p = g[r];
#pragma unroll
        for (int n = 0; n < N; ++n) p *= u[n][r];
        x += p;
    }
    return x;
}

// contraction kinds of the per-entry kernels
constexpr int kReuse = 0;  // single pass with reuse (above)
constexpr int kNaive = 1;  // ablation: no reuse
constexpr int kCP = 2;     // hyper-diagonal core
constexpr int kMfma32 = 3; // dense part on the matrix cores, FP32 operands (mfma.hpp)
constexpr int kMfma16 = 4; // dense part on the matrix cores, BF16 operands, FP32 sums
constexpr bool is_mx(int ct) { return ct == kMfma32 || ct == kMfma16; }

template <int CT, int N, int JP, typename T, typename GP>
S3_DEV void contract_any(GP G, const T (&u)[N][JP], T (&w)[N][JP], T &xhat) {
    if constexpr (CT == kCP) contract_cp<N, JP, T>(G, u, w, xhat);
    else if constexpr (CT == kNaive) contract_naive<N, JP, T>(G, u, w, xhat);
    else contract<N, JP, T>(G, u, w, xhat);
}

template <int CT, int N, int JP, typename T, typename GP> S3_DEV T predict_any(GP G, const T (&u)[N][JP]) {
    if constexpr (CT == kCP) return predict_cp<N, JP, T>(G, u);
    else return predict<N, JP, T>(G, u);
}

// curvature of x~ in the core values: prod_n |u_n|^2 (the squared norm of
// u^(1) o ... o u^(N)), or for a hyper-diagonal core sum_r prod_n u_n[r]^2
template <int CT, int N, int JP, typename T> S3_DEV T core_curv(const T (&u)[N][JP]) {
    if constexpr (CT == kCP) {
        T s = T(0);
#pragma unroll
        for (int r = 0; r < JP; ++r) {
            T p = T(1);
#pragma unroll
            for (int n = 0; n < N; ++n) p *= u[n][r] * u[n][r];
            s += p;
        }
        return s;
    } else {
        T p = T(1);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            T uu = T(0);
#pragma unroll
            for (int k = 0; k < JP; ++k) uu = fmaT(u[n][k], u[n][k], uu);
            p *= uu;
        }
        return p;
    }
}

}  // namespace s3
