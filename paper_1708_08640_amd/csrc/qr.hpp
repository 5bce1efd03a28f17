// Orthogonalisation of the factors after training (Algorithm 1, closing
// step): U^(n) = Q R, then U^(n) <- Q, G <- G x_n R and, for every coupled
// matrix on mode n, V <- V R^T.  The model's predictions are unchanged.
//
// The QR of a tall-skinny I x J factor (J <= 16) is CholeskyQR2: the Gram
// matrix A = U^T U is summed in FP64 over fixed row chunks (one workgroup
// each, added in chunk order), factored A = R^T R on one lane (R upper with a
// positive diagonal, so Q is unique), and U <- U R^-1 row by row in FP64; a
// second pass restores orthogonality lost to rounding and R = R2 R1.
//   k_gram          per-chunk Gram partials
//   k_chol          chunk sum, Cholesky, R^-1, running product R <- R_pass R
//   k_apply_rinv    U <- U R^-1
//   k_core_mode_mul G <- G x_n R (out of place)
//   k_rows_times_rt V <- V R^T
#pragma once
#include "common.hpp"

namespace s3 {

constexpr int kQrBlocks = 512;
constexpr int kQrJ = 16;  // largest rank
constexpr int kQrRows = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_gram(const T *__restrict__ U, int64_t I, int J, double *__restrict__ part) {
    __shared__ double s_rows[kQrRows][kQrJ + 1];
    const int tid = threadIdx.x, j = tid / kQrJ, k = tid % kQrJ;
    const int64_t chunk = (I + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = (r0 + chunk < I) ? r0 + chunk : I;
    double acc = 0.0;
    for (int64_t b0 = r0; b0 < r1; b0 += kQrRows) {
        const int cnt = (int)((r1 - b0 < kQrRows) ? r1 - b0 : kQrRows);
        __syncthreads();
        for (int x = tid; x < kQrRows * J; x += blockDim.x) {
            const int t = x / J, c = x - t * J;
            s_rows[t][c] = (t < cnt) ? (double)U[(b0 + t) * J + c] : 0.0;
        }
        __syncthreads();
        if (j < J && k < J)
            for (int t = 0; t < cnt; ++t) acc = fma(s_rows[t][j], s_rows[t][k], acc);
    }
    part[(int64_t)blockIdx.x * kQrJ * kQrJ + tid] = acc;
}

// R, Rinv, Rtot: kQrJ x kQrJ row-major.  first != 0: Rtot <- R, else
// Rtot <- R Rtot.  A factor that is not numerically full rank sets *flag and
// leaves R = I.
static __global__ __launch_bounds__(256) void k_chol(const double *__restrict__ part, int nb, int J, double *__restrict__ R,
                                              double *__restrict__ Rinv, double *__restrict__ Rtot, int first,
                                              int32_t *__restrict__ flag) {
    __shared__ double A[kQrJ][kQrJ];
    __shared__ double Rs[kQrJ][kQrJ];
    const int tid = threadIdx.x, j = tid / kQrJ, k = tid % kQrJ;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * kQrJ * kQrJ + tid];
    A[j][k] = s;
    Rs[j][k] = 0.0;
    __syncthreads();
    if (tid == 0) {
        bool ok = true;
        for (int i = 0; i < J && ok; ++i) {
            double d = A[i][i];
            for (int q = 0; q < i; ++q) d -= Rs[q][i] * Rs[q][i];
            if (!(d > 0.0) || !isfinite(d)) { ok = false; break; }
            const double rii = sqrt(d);
            Rs[i][i] = rii;
            for (int c = i + 1; c < J; ++c) {
                double v = A[i][c];
                for (int q = 0; q < i; ++q) v -= Rs[q][i] * Rs[q][c];
                Rs[i][c] = v / rii;
            }
        }
        if (!ok) {
            *flag = 1;
            for (int a = 0; a < kQrJ; ++a)
                for (int c = 0; c < kQrJ; ++c) Rs[a][c] = (a == c) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    // inverse of the upper-triangular R by back substitution, column k per lane
    if (tid < J) {
        const int c = tid;
        double x[kQrJ];
        for (int i = J - 1; i >= 0; --i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int q = i + 1; q < J; ++q) v -= Rs[i][q] * x[q];
            x[i] = (i <= c) ? v / Rs[i][i] : 0.0;
        }
        for (int i = 0; i < kQrJ; ++i) Rinv[i * kQrJ + c] = (i < J) ? x[i] : 0.0;
    }
    // Rtot <- R Rtot (row j, column k per lane)
    double t = 0.0;
    if (j < J && k < J) {
        if (first) {
            t = Rs[j][k];
        } else {
            for (int q = 0; q < J; ++q) t += Rs[j][q] * Rtot[q * kQrJ + k];
        }
    }
    __syncthreads();  // every lane has read the old Rtot
    Rtot[j * kQrJ + k] = t;
    R[j * kQrJ + k] = Rs[j][k];
}

template <typename T>
__global__ __launch_bounds__(256) void k_apply_rinv(T *__restrict__ U, int64_t I, int J,
                                                    const double *__restrict__ Rinv) {
    __shared__ double s[kQrJ][kQrJ];
    s[threadIdx.x / kQrJ][threadIdx.x % kQrJ] = Rinv[threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I; i += (int64_t)gridDim.x * blockDim.x) {
        T *row = U + i * J;
        double u[kQrJ];
#pragma unroll
        for (int c = 0; c < kQrJ; ++c) u[c] = (c < J) ? (double)row[c] : 0.0;
#pragma unroll
        for (int c = 0; c < kQrJ; ++c) {
            if (c >= J) break;
            double v = 0.0;
#pragma unroll
            for (int q = 0; q <= c; ++q) v = fma(u[q], s[q][c], v);
            row[c] = (T)v;
        }
    }
}

// Gout = Gin x_n R over the core J_0 x .. x J_{N-1} (row-major, last index
// fastest): Gout[.., i, ..] = sum_k R[i][k] Gin[.., k, ..]
template <typename T>
__global__ void k_core_mode_mul(const T *__restrict__ Gin, T *__restrict__ Gout, int N, int J0, int J1, int J2,
                                int J3, int n, const double *__restrict__ R) {
    const int Js[4] = {J0, J1, J2, J3};
    int K = 1, stride = 1;
    for (int q = 0; q < N; ++q) K *= Js[q];
    for (int q = N - 1; q > n; --q) stride *= Js[q];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < K; j += gridDim.x * blockDim.x) {
        const int i = (j / stride) % Js[n];
        const int base = j - i * stride;
        double v = 0.0;
        for (int k = 0; k < Js[n]; ++k) v = fma(R[i * kQrJ + k], (double)Gin[base + k * stride], v);
        Gout[j] = (T)v;
    }
}

// V <- V R^T: v_new[i] = sum_k v[k] R[i][k]
template <typename T>
__global__ __launch_bounds__(256) void k_rows_times_rt(T *__restrict__ V, int64_t rows, int J,
                                                       const double *__restrict__ R) {
    __shared__ double s[kQrJ][kQrJ];
    s[threadIdx.x / kQrJ][threadIdx.x % kQrJ] = R[threadIdx.x];
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        T *row = V + r * J;
        double v[kQrJ];
#pragma unroll
        for (int c = 0; c < kQrJ; ++c) v[c] = (c < J) ? (double)row[c] : 0.0;
#pragma unroll
        for (int i = 0; i < kQrJ; ++i) {
            if (i >= J) break;
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < kQrJ; ++k) t = fma(v[k], s[i][k], t);
            row[i] = (T)t;
        }
    }
}

}  // namespace s3
