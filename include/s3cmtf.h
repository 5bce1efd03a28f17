/*
 * s3cmtf.h -- C ABI of the MI355X (gfx950) library for sparse coupled
 * matrix-tensor factorisation with a Tucker model trained by per-entry
 * stochastic gradient descent (S^3CMTF, Choi, Jang and Kang, arXiv
 * 1708.08640).
 *
 * Model (Section 3.2, Eq 4 and Definition 1).  An order-N tensor X
 * (I_1 x ... x I_N) with observed entries Omega_X is approximated by a core
 * G (J_1 x ... x J_N) and factors U^(n) (I_n x J_n):
 *     x~_alpha = sum_j g_j prod_n u^(n)_{i_n j_n}.
 * Each coupled matrix Y_m (I_{c_m} x K_m), observed on Omega_{Y_m}, is
 * approximated by U^(c_m) V_m^T with its own factor V_m (K_m x J_{c_m}).
 *
 * Objective (Eq 7) and per-entry gradients (Eq 8) are those of the paper;
 * the library runs them on one GPU in two modes:
 *   S3_DET_MINIBATCH  the item order is cut into batches of `batch` items;
 *                     every gradient of a batch is taken at the batch-start
 *                     values, gradients are summed per parameter in a fixed
 *                     order and applied once (batch = 1 is Algorithm 1 with
 *                     one worker).  Bitwise reproducible run to run.
 *   S3_LOCKFREE       lock-free parallel SGD (Section 3.3): the items of a
 *                     round (s3_desc.round_items) are in flight at once; a
 *                     factor row is updated without locks by a plain
 *                     read-modify-write as soon as its entry is processed,
 *                     so the write order differs from run to run.  The
 *                     most frequent rows of each mode and coupled factor
 *                     (s3_desc.hot_rows) and the core are instead summed
 *                     over the round and moved once, damped (see
 *                     s3_desc.damping).
 *
 * Layouts (device memory unless stated; all indices 0-based, int32):
 *   tensor entries   idx[n * nnz + e] = mode-n index of entry e (SoA)
 *   values           val[e], in the compute type (double for S3_F64,
 *                    float otherwise)
 *   factor U[n]      I_n x J_n row-major
 *   core G           J_1 x ... x J_N row-major (last index fastest)
 *   coupled V[m]     K_m x J_{c_m} row-major
 *   matrix entries   row[e] (index into mode c_m), col[e] (into V_m), val[e]
 *   item ids         0..nX-1 are the training tensor entries, then the
 *                    entries of matrix 0, matrix 1, ... back to back.
 *
 * Ownership: the caller allocates every device buffer (inputs, parameters
 * and one workspace) and keeps it alive until s3_plan_destroy.  The library
 * allocates no device memory.  Parameters are updated in place.
 *
 * Streams: every call that touches the device takes a hipStream_t (passed as
 * void*) and enqueues on it.  s3_bind, s3_loss, s3_rmse and s3_export
 * synchronise that stream; the others are asynchronous.  An asynchronous
 * device error surfaces at the next synchronising call as S3_ERR_HIP.
 *
 * Errors: every call returns an s3_status; no exception crosses the ABI.
 * A failed call leaves the plan's state unchanged except where stated and
 * records a message readable with s3_last_error.  A plan is not thread safe;
 * distinct plans are independent.
 */
#ifndef S3CMTF_H
#define S3CMTF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define S3_MAX_ORDER 4
#define S3_MAX_MATRICES 4

typedef int32_t s3_status;
enum {
    S3_OK = 0,
    S3_ERR_INVALID_ARG = -1,  /* null pointer, negative size, bad enum     */
    S3_ERR_INDEX_RANGE = -2,  /* an entry index outside its mode / matrix  */
    S3_ERR_UNSUPPORTED = -3,  /* order, rank or dtype outside what is built */
    S3_ERR_NONFINITE = -4,    /* loss or RMSE not finite (diverged)        */
    S3_ERR_HIP = -5,          /* a HIP runtime call failed                 */
    S3_ERR_WORKSPACE = -6,    /* workspace null or smaller than required   */
    S3_ERR_STATE = -7         /* call out of order (e.g. epoch before bind) */
};

enum { S3_F64 = 0, S3_F32 = 1, S3_BF16 = 2 };          /* s3_desc.dtype */
enum { S3_DET_MINIBATCH = 0, S3_LOCKFREE = 1 };         /* s3_epoch mode */
enum { S3_DAMP_NONE = 0, S3_DAMP_CURVATURE = 1 };       /* s3_desc.damping */

/* Problem and hyper-parameters.  dims/rank/mat_* beyond order / n_mat are
 * ignored.  Hyper-parameters follow Section 4.1 ("Parameters"): the
 * learning rate of epoch t is eta0 / (1 + mu t) (Algorithm 1); lambda_reg
 * regularises factors and core, lambda_m weighs the coupled matrices
 * (Eq 7).
 *
 * damping: S3_DAMP_NONE sums the gradients that land on one parameter
 * block (a factor row, a coupled-factor row or the whole core) and applies
 * -eta * sum.  S3_DAMP_CURVATURE divides that step by max(1, (N+1) eta L),
 * where L sums, over the same contributions, the curvature of the entry's
 * squared error along the block (|w_n|^2 for a tensor row, prod_n |u^(n)|^2
 * for the core -- sum_r prod_n u^(n)_r^2 for a hyper-diagonal core --,
 * lambda_m |v|^2 and lambda_m |u|^2 for a matrix entry) plus
 * the regularisation weight.  A block touched once with (N+1) eta L <= 1
 * moves exactly as one SGD step; a block that many concurrent entries touch
 * can no longer overshoot (N+1 bounds the joint step of the N rows and the
 * core of one entry).  The lock-free mode always damps.  (Not in the paper:
 * a reading needed to keep thousands of concurrent updates of power-law-hot
 * rows stable.)                                                            */
/* Per-entry contraction (s3_desc.contraction). */
#define S3_CONTRACT_REUSE 0
#define S3_CONTRACT_NAIVE 1
#define S3_CONTRACT_MATRIX 2  /* the dense part on the matrix cores, 32
                                 entries at a time: 3-way, the mode products
                                 G x_1 u^(1) and G x_3 u^(3) as (J^2 x J) .
                                 (J x 32) products; 4-way, G x_1 u^(1) x_2 u^(2)
                                 and G x_3 u^(3) x_4 u^(4) as (J^2 x J^2) .
                                 (J^2 x 32) products whose columns are the
                                 entries' Khatri-Rao products (Definition 1).
                                 The rest of Eq (8)'s contractions reuse them
                                 on the vector units (Algorithm 3's reuse of
                                 partial products, without its divisions); the
                                 core gradient of each 256-entry tile runs on
                                 the matrix cores too.  Operands FP32 (S3_F32)
                                 or BF16 (S3_BF16), sums in FP32.  Built for
                                 3-way tensors with padded rank 16 (ranks
                                 13..16) and 4-way tensors with padded rank 8
                                 (ranks 5..8)                                 */

/* Core structure (s3_desc.core_kind). */
#define S3_CORE_TUCKER 0   /* dense core J_1 x ... x J_N (Eq 4)             */
#define S3_CORE_CP 1       /* hyper-diagonal core (the CP special case of
                              Section 3): every J_n equals J and G holds the
                              J diagonal values; s3_orthogonalize does not
                              apply                                          */

typedef struct {
    int32_t order;                       /* N: 3 or 4                        */
    int32_t n_mat;                       /* M: 0..S3_MAX_MATRICES            */
    int64_t dims[S3_MAX_ORDER];          /* I_n                              */
    int32_t rank[S3_MAX_ORDER];          /* J_n                              */
    int32_t mat_mode[S3_MAX_MATRICES];   /* c_m, coupled tensor mode         */
    int64_t mat_cols[S3_MAX_MATRICES];   /* K_m                              */
    int32_t dtype;                       /* S3_F64, S3_F32, or S3_BF16: FP32
                                            values and parameters (the master
                                            copies) whose contraction operands
                                            are rounded to BF16 (round to
                                            nearest even) as they are read;
                                            needs S3_CONTRACT_MATRIX.  Loss,
                                            RMSE, the row updates and the core
                                            update stay FP32                  */
    int32_t damping;                     /* S3_DAMP_*                        */
    double eta0, mu, lambda_reg, lambda_m;
    int64_t batch;                       /* det mode: items per batch (>= 1) */
    int64_t round_items;                 /* lock-free: items per round (>= 1) */
    uint64_t seed;                       /* lock-free tile shuffle seed      */
    int32_t hot_rows;                    /* lock-free: rows per mode kept in the
                                            per-round hot tables (0: as many as
                                            the LDS budget allows, <= 256; -1:
                                            none, every row is updated at once) */
    int32_t contraction;                 /* S3_CONTRACT_REUSE (default; the
                                            single pass on the vector units),
                                            S3_CONTRACT_NAIVE: the per-entry
                                            contraction without reuse of partial
                                            products (Algorithm 2's cost, an
                                            ablation of Lemma 4; N = 3 with
                                            J <= 4 or J = 10, N = 4 with J <= 2,
                                            else S3_ERR_UNSUPPORTED), or
                                            S3_CONTRACT_MATRIX (above; FP32 or
                                            BF16 only, Tucker core only)      */
    int32_t core_kind;                   /* S3_CORE_TUCKER (default) or
                                            S3_CORE_CP (then every rank must be
                                            equal, else S3_ERR_INVALID_ARG, and
                                            contraction must be REUSE)        */
} s3_desc;

/* Device buffers handed to s3_bind.  Values and parameters are `double` for
 * S3_F64 and `float` for S3_F32 and S3_BF16.                               */
typedef struct {
    const int32_t *x_idx;  const void *x_val;  int64_t x_nnz;   /* training */
    const int32_t *t_idx;  const void *t_val;  int64_t t_nnz;   /* held-out */
    const int32_t *y_row[S3_MAX_MATRICES];
    const int32_t *y_col[S3_MAX_MATRICES];
    const void    *y_val[S3_MAX_MATRICES];
    int64_t        y_nnz[S3_MAX_MATRICES];
    void *U[S3_MAX_ORDER];
    void *G;
    void *V[S3_MAX_MATRICES];
    /* det mode: the item order, a permutation of 0..n_items-1 (n_items =
     * x_nnz + sum y_nnz), int32.  May be null if det mode is never run
     * (s3_backward then sums in the storage order).                      */
    const int32_t *order;
} s3_buffers;

typedef struct s3_plan s3_plan;

/* Human-readable name of a status code (static storage). */
const char *s3_status_string(s3_status st);

/* Copy the plan's last error message into buf (always NUL-terminated). */
s3_status s3_last_error(const s3_plan *plan, char *buf, size_t len);

/* Validate `desc` and create a plan (host memory only).
 * S3_ERR_UNSUPPORTED if order is not 3 or 4, a rank exceeds what the
 * kernels are built for, or the dtype is unknown.                       */
s3_status s3_plan_create(const s3_desc *desc, s3_plan **plan);

/* Free the plan (host memory only; device buffers stay the caller's). */
s3_status s3_plan_destroy(s3_plan *plan);

/* Bytes of device workspace s3_bind needs for these entry counts
 * (x_nnz, t_nnz, y_nnz[M]), with the det-mode structures included.  Host
 * only.  S3_ERR_UNSUPPORTED if the det-mode structures of these counts do
 * not fit their 32-bit fields (a batch's scratch beyond 2^32 values, or
 * batches x (M + 1) beyond 2^32).                                         */
s3_status s3_workspace_size(const s3_plan *plan, int64_t x_nnz, int64_t t_nnz,
                            const int64_t *y_nnz, size_t *bytes);

/* Bind buffers and a workspace of ws_bytes at d_ws (device).  On the device
 * it checks every index against its mode / matrix size (S3_ERR_INDEX_RANGE
 * and nothing bound if one is out of range), builds the counts
 * |Omega_X^{n,i}| and |Omega_Y^{2,k}| of Eq (7), and, when buf->order is
 * given, the fixed per-batch reduction order of det mode (S3_ERR_UNSUPPORTED,
 * before any device access, if it would overflow its 32-bit fields; see
 * s3_workspace_size).  S3_ERR_WORKSPACE if ws_bytes is too small.
 * The plan keeps the buffers' addresses: they stay the caller's, must stay
 * allocated until the plan is destroyed, and the index buffers must not
 * change while bound (they are range-checked only here; the parameters are
 * updated in place).  Synchronises `stream`.                              */
s3_status s3_bind(s3_plan *plan, const s3_buffers *buf, void *d_ws, size_t ws_bytes,
                  void *stream);

/* One epoch (Algorithm 1's inner loop over all training items) at learning
 * rate eta0 / (1 + mu * epoch).  mode: S3_DET_MINIBATCH or S3_LOCKFREE.
 * Asynchronous.                                                           */
s3_status s3_epoch(s3_plan *plan, int32_t epoch, int32_t mode, void *stream);

/* Det mode only: run batches [first, first + count) of the item order at
 * learning rate eta (for step-by-step checks).  Asynchronous.             */
s3_status s3_det_batches(s3_plan *plan, int64_t first, int64_t count, double eta,
                         void *stream);

/* Objective of Eq (7) over the training items: out[0] = f, out[1] = f_t,
 * out[2] = f_m (host doubles).  Synchronous; S3_ERR_NONFINITE if f is not
 * finite.                                                                  */
s3_status s3_loss(s3_plan *plan, double *out, void *stream);

/* Held-out RMSE, sqrt(mean over test entries of (x - x~)^2) (Section 4.1,
 * "Measure"); 0 when the plan was bound without held-out entries.
 * Synchronous; S3_ERR_NONFINITE if not finite.                           */
s3_status s3_rmse(s3_plan *plan, double *out, void *stream);

/* Forward of the prediction map, the Tucker reconstruction of Eq (4):
 * x~ = sum over core positions j of g_j * prod_n u^(n)_{i_n, j_n}, for nnz
 * entries idx (device, SoA: idx[n * nnz + e] is entry e's mode-n index) into
 * xhat (device, nnz values in the compute type: FP64 plans FP64, FP32 and
 * BF16-operand plans FP32).  The caller owns both buffers.  The indices are
 * checked against their modes first (S3_ERR_INDEX_RANGE, nothing written),
 * which synchronises `stream`; the prediction itself is enqueued on it.    */
s3_status s3_predict(s3_plan *plan, const int32_t *idx, int64_t nnz, void *xhat,
                     void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc; not code under HIP graph capture, since
 * the index check synchronises the stream): the same
 * result as s3_predict, bitwise, with its working memory (the index-check
 * flag and the zero-padded core, at most 64 KiB) taken from a static array
 * in the library's device code instead of the plan's workspace.  Allocates
 * nothing.  Each GPU holds one copy of that array until the process ends;
 * it is set up by s3_bind on that device.  Calls that overlap on one GPU (on
 * different streams, or from different plans) share it and race: serialise
 * them.  S3_ERR_WORKSPACE if the plan's padded core does not fit.
 * Synchronises `stream` (index check), like s3_predict.                   */
s3_status s3_predict_noalloc(s3_plan *plan, const int32_t *idx, int64_t nnz, void *xhat,
                             void *stream);

/* Forward of coupled matrix m: yhat[e] = u^(c_m)_{row[e]} . v_{col[e]} for nnz
 * entries (row, col, yhat on the device; yhat in the compute type).
 * Asynchronous.                                                           */
s3_status s3_predict_matrix(s3_plan *plan, int32_t m, const int32_t *row, const int32_t *col,
                            int64_t nnz, void *yhat, void *stream);

/* Adjoint (backward) of the prediction map over the bound training entries:
 * given gx[e] = dL/dx~_e (device, compute type, x_nnz) and gy[m][e] =
 * dL/dy^_e for each coupled matrix (may be null for a matrix with no
 * upstream gradient), write
 *   dU[n] = sum_e gx[e] [G x_{-n} {u}_e]  (+ sum over matrix entries gy v)
 *   dG    = sum_e gx[e] (u^(1)_e o ... o u^(N)_e)
 *   dV[m] = sum_e gy[m][e] u^(c)_r
 * (device, shaped like the parameters, overwritten).  The contraction is
 * the one of Eq (8); summation order is fixed (deterministic): every row's
 * contributions are summed in the bound item order, or, on a plan bound
 * without one, in the storage order (training entries, then each matrix's
 * entries).  Such a plan builds those reduction structures on its first
 * call, in the part of the bound workspace the det structures would use:
 * that call synchronises `stream` and needs the workspace that
 * s3_workspace_size reports (S3_ERR_WORKSPACE if a smaller one was bound,
 * S3_ERR_UNSUPPORTED past its 32-bit limits).  Det epochs still need an
 * item order.  Otherwise asynchronous.                                     */
s3_status s3_backward(s3_plan *plan, const void *gx, const void *const *gy,
                      void *const *dU, void *dG, void *const *dV, void *stream);

/* Copy a parameter to host memory as float64: which = 0 -> U[index],
 * 1 -> G, 2 -> V[index].  bytes must equal rows * cols * 8.  Synchronous. */
s3_status s3_export(s3_plan *plan, int32_t which, int32_t index, double *host_dst,
                    size_t bytes, void *stream);

/* The inverse of s3_export, for checkpoint and resume: copy a parameter from
 * host memory (float64, the caller's, row-major as exported) into the bound
 * plan's parameter buffer; which/index/bytes as for s3_export.  FP32 and
 * BF16-operand plans store each value rounded to the nearest FP32 (their
 * masters).  A value that is not finite gives S3_ERR_NONFINITE and nothing
 * is written.  Every later call reads the new values (derived copies of the
 * core are rebuilt at the start of each call).  The learning rate depends
 * only on the epoch index passed to s3_epoch (Algorithm 1's schedule), so a
 * det run resumed by importing every parameter exported after epoch e and
 * continuing with epoch e + 1 reproduces the uninterrupted run bitwise.
 * Synchronous.                                                            */
s3_status s3_import(s3_plan *plan, int32_t which, int32_t index, const double *host_src,
                    size_t bytes, void *stream);

/* Orthogonalise the bound parameters in place (Algorithm 1, closing step):
 * every factor U^(n) = Q R becomes Q (orthonormal columns), the core becomes
 * G x_n R for every mode n, and every coupled V_m becomes V_m R^(c_m)T, so
 * all predictions are unchanged.  QR is CholeskyQR2 with the Gram matrix,
 * Cholesky factor and R^-1 in FP64 (R has a positive diagonal, so Q is
 * unique).  Needs J_n <= min(16, I_n) (else S3_ERR_UNSUPPORTED); a factor
 * that is not numerically full rank gives S3_ERR_NONFINITE and is left
 * partly transformed.  Synchronous.                                        */
s3_status s3_orthogonalize(s3_plan *plan, void *stream);

/* Fill every bound parameter (U^(n), G, V_m) with independent N(0, sigma^2)
 * values on the device, the random initialisation of Algorithm 1; callers
 * may instead write their own initial values into the buffers they bound.
 * Counter-based: value 2i (and 2i + 1) of parameter q (q = n for U^(n),
 * N for G, N + 1 + m for V_m) is the Box-Muller pair, in FP64, of the 53-bit
 * uniforms of counters key_q + 2i and key_q + 2i + 1 passed through
 * SplitMix64's output function, with key_q = that function applied to
 * seed + (q + 1) * 0x9E3779B97F4A7C15 (u1 = (bits + 1) 2^-53 in (0, 1], u2 =
 * bits 2^-53 in [0, 1); element 2i = sigma sqrt(-2 ln u1) cos(2 pi u2),
 * element 2i + 1 the same with sin).  The result does not depend on the
 * launch shape.  Needs s3_bind (else S3_ERR_STATE); sigma must be finite and
 * >= 0 (else S3_ERR_INVALID_ARG).  Asynchronous on stream.                 */
s3_status s3_init_params(s3_plan *plan, uint64_t seed, double sigma, void *stream);

/* Turn per-launch timing of the dominant kernel (the tensor-entry kernel of
 * the epoch's mode) on or off; off by default.  When on, each such launch
 * carries a pair of timing-only HIP events (no system-scope fence) that the
 * dispatch itself stamps at its start and end (hipExtLaunchKernelGGL).     */
s3_status s3_set_profiling(s3_plan *plan, int32_t on);

/* After s3_epoch: with profiling on, the summed duration in milliseconds of
 * the dominant kernel's launches and their count; with profiling off, the
 * whole epoch's duration and the number of batches / rounds.  Waits for the
 * epoch to finish.                                                          */
s3_status s3_last_epoch_profile(const s3_plan *plan, double *kernel_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* S3CMTF_H */
