/*
 * FP64 CPU oracle for sparse coupled Tucker factorisation by per-entry SGD
 * (S^3CMTF, Choi, Jang and Kang, arXiv 1708.08640).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header
 * or constant with the HIP library, and the HIP library never calls it.
 *
 * Everything is double precision, sequential, with plain loops that follow
 * the paper's definitions; no blocking, fusion or reordering beyond what the
 * definitions state.
 *
 * Layouts (all 0-based):
 *   tensor entries  idx[n * nnz + e] (mode n of entry e), val[e]
 *   factor U[n]     I_n x J_n, row-major (row i at U[n] + i * J_n)
 *   core G          J_1 x ... x J_N, row-major: the LAST core index varies
 *                   fastest, flat index j = ((j_1 * J_2 + j_2) * J_3 + j_3)...
 *   coupled factor  V[m]: K_m x J_{c_m}, row-major
 *   matrix entries  row[e] (index into mode c_m), col[e] (index into V[m])
 *   item ids        0..nX-1 are training tensor entries; then matrix 0's
 *                   entries, matrix 1's entries, ... in order.
 *
 * Readings where the paper is silent or inconsistent:
 *   - core regulariser per tensor entry is (lambda_reg / |Omega_X|) G, the
 *     form of Eq (8) and Algorithm 2 (the efficient-gradient lemma drops the
 *     1/|Omega_X| factor, which would make it disagree with the objective);
 *   - counts |Omega_X^{n,i}| and |Omega_Y^{2,k}| are taken over the training
 *     entries; a row with count 0 is never touched;
 *   - every gradient of one entry is evaluated at the pre-update values
 *     (simultaneous update of the rows and the core);
 *   - the core is updated after every tensor entry (one worker, P = 1).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 8
#define OR_MAXM 8

typedef struct {
    int32_t N;
    int32_t M;
    int64_t dims[OR_MAXN];
    int32_t J[OR_MAXN];
    double *U[OR_MAXN];
    double *G;
    int32_t mode[OR_MAXM];
    int64_t cols[OR_MAXM];
    double *V[OR_MAXM];
    int32_t cp;     /* 1: hyper-diagonal core (the CP special case of the
                       model, Section 3's S^3CMTF-CP): every J_n equals J, G
                       holds the J diagonal values g_r = G[r, .., r], and the
                       core's other entries are structurally zero */
} or_model;

typedef struct {
    int64_t nnz;
    const int32_t *idx;
    const double *val;
} or_tensor;

typedef struct {
    int64_t nnz;
    const int32_t *row;
    const int32_t *col;
    const double *val;
} or_matrix;

typedef struct {
    int64_t nX;                 /* |Omega_X| over the training entries */
    int64_t *cnt[OR_MAXN];      /* cnt[n][i] = |Omega_X^{n,i}|          */
    int64_t *cntV[OR_MAXM];     /* cntV[m][k] = |Omega_Y^{2,k}|         */
} or_counts;

typedef struct {
    double lambda_reg;
    double lambda_m;
} or_hyper;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */

/* number of stored core values: prod J_n, or J for a hyper-diagonal core */
static int64_t core_size(const or_model *md)
{
    if (md->cp) return md->J[0];
    int64_t K = 1;
    for (int n = 0; n < md->N; ++n) K *= md->J[n];
    return K;
}

/* decode a stored core index into its position (j_1..j_N) in the core: a
 * row-major flat index, or for a hyper-diagonal core the position (r..r).
 * Every sum over the core below runs over the stored values, so the CP
 * model needs no other change: its entries off the diagonal are zero.      */
static void decode(const or_model *md, int64_t flat, int32_t *jj)
{
    if (md->cp) {
        for (int n = 0; n < md->N; ++n) jj[n] = (int32_t)flat;
        return;
    }
    for (int n = md->N - 1; n >= 0; --n) {
        jj[n] = (int32_t)(flat % md->J[n]);
        flat /= md->J[n];
    }
}

static const double *urow(const or_model *md, int n, int64_t i)
{
    return md->U[n] + i * md->J[n];
}

static int64_t rank_sum(const or_model *md)
{
    int64_t s = 0;
    for (int n = 0; n < md->N; ++n) s += md->J[n];
    return s;
}

/* The positions (j_1..j_N) of every stored core value, decoded once per call
 * instead of once per use: pos[j * N + n] = j_n of stored value j.  Only the
 * index arithmetic moves; every sum and product below is formed in the same
 * order as with decode() in the loop.                                      */
typedef struct {
    int64_t K;
    int N;
    int32_t *pos;
} or_cpos;

static int cpos_make(const or_model *md, or_cpos *t)
{
    t->K = core_size(md);
    t->N = md->N;
    t->pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t->K * t->N));
    if (!t->pos) return 0;
    for (int64_t j = 0; j < t->K; ++j) decode(md, j, t->pos + j * t->N);
    return 1;
}

static void cpos_free(or_cpos *t)
{
    free(t->pos);
    t->pos = NULL;
}

/* the N factor rows of a tensor entry */
static void entry_rows(const or_model *md, const int32_t *rows, const double **ur)
{
    for (int n = 0; n < md->N; ++n) ur[n] = urow(md, n, rows[n]);
}

/* ------------------------------------------------------------------ */
/* Counts |Omega_X^{n,i}| (Table 2 and the rewritten objective, Eq 7)  */

void or_counts_build(const or_model *md, const or_tensor *X, int32_t M,
                     const or_matrix *Y, or_counts *c)
{
    c->nX = X->nnz;
    for (int n = 0; n < md->N; ++n) {
        memset(c->cnt[n], 0, sizeof(int64_t) * (size_t)md->dims[n]);
        for (int64_t e = 0; e < X->nnz; ++e) c->cnt[n][X->idx[n * X->nnz + e]] += 1;
    }
    for (int m = 0; m < M; ++m) {
        memset(c->cntV[m], 0, sizeof(int64_t) * (size_t)md->cols[m]);
        for (int64_t e = 0; e < Y[m].nnz; ++e) c->cntV[m][Y[m].col[e]] += 1;
    }
}

/* ------------------------------------------------------------------ */
/* Tucker prediction, Eq (4): x~ = sum_j g_j prod_n u^(n)_{i_n j_n}     */

/* Order-3 and order-4 dense cores with the core positions as loop counters
 * (stored index j = ((j_1 J_2 + j_2) J_3 + j_3) J_4 + j_4, the row-major
 * order above): the same products, multiplied in mode order, and the same
 * sums, added in increasing j, as the general loops over the table.       */
static int nested(const or_model *md)
{
    return !md->cp && (md->N == 3 || md->N == 4);
}

static double predict_nested(const or_model *md, const double *const *ur)
{
    const double *G = md->G, *a = ur[0], *b = ur[1], *c = ur[2];
    const int J1 = md->J[0], J2 = md->J[1], J3 = md->J[2];
    double acc = 0.0;
    int64_t j = 0;
    if (md->N == 3) {
        for (int j1 = 0; j1 < J1; ++j1)
            for (int j2 = 0; j2 < J2; ++j2)
                for (int j3 = 0; j3 < J3; ++j3, ++j) {
                    double p = G[j];
                    p *= a[j1]; p *= b[j2]; p *= c[j3];
                    acc += p;
                }
        return acc;
    }
    const double *d = ur[3];
    const int J4 = md->J[3];
    for (int j1 = 0; j1 < J1; ++j1)
        for (int j2 = 0; j2 < J2; ++j2)
            for (int j3 = 0; j3 < J3; ++j3)
                for (int j4 = 0; j4 < J4; ++j4, ++j) {
                    double p = G[j];
                    p *= a[j1]; p *= b[j2]; p *= c[j3]; p *= d[j4];
                    acc += p;
                }
    return acc;
}

/* w_n (into w, J_1 + ... + J_N values, overwritten) and, when gG is not
 * null, the core gradient -e prod_n u^(n) + reg_core G, in one pass        */
static void loo_nested(const or_model *md, const double *const *ur, double *w, double e,
                       double reg_core, double *gG)
{
    const double *G = md->G, *a = ur[0], *b = ur[1], *c = ur[2];
    const int J1 = md->J[0], J2 = md->J[1], J3 = md->J[2];
    const int J4 = md->N == 4 ? md->J[3] : 1;
    double *w1 = w, *w2 = w1 + J1, *w3 = w2 + J2, *w4 = w3 + J3;
    for (int k = 0; k < J1 + J2 + J3 + (md->N == 4 ? J4 : 0); ++k) w[k] = 0.0;
    int64_t j = 0;
    if (md->N == 3) {
        for (int j1 = 0; j1 < J1; ++j1)
            for (int j2 = 0; j2 < J2; ++j2)
                for (int j3 = 0; j3 < J3; ++j3, ++j) {
                    const double g = G[j];
                    double p;
                    p = g; p *= b[j2]; p *= c[j3]; w1[j1] += p;
                    p = g; p *= a[j1]; p *= c[j3]; w2[j2] += p;
                    p = g; p *= a[j1]; p *= b[j2]; w3[j3] += p;
                    if (gG) {
                        p = 1.0; p *= a[j1]; p *= b[j2]; p *= c[j3];
                        gG[j] = -e * p + reg_core * g;
                    }
                }
        return;
    }
    const double *d = ur[3];
    for (int j1 = 0; j1 < J1; ++j1)
        for (int j2 = 0; j2 < J2; ++j2)
            for (int j3 = 0; j3 < J3; ++j3)
                for (int j4 = 0; j4 < J4; ++j4, ++j) {
                    const double g = G[j];
                    double p;
                    p = g; p *= b[j2]; p *= c[j3]; p *= d[j4]; w1[j1] += p;
                    p = g; p *= a[j1]; p *= c[j3]; p *= d[j4]; w2[j2] += p;
                    p = g; p *= a[j1]; p *= b[j2]; p *= d[j4]; w3[j3] += p;
                    p = g; p *= a[j1]; p *= b[j2]; p *= c[j3]; w4[j4] += p;
                    if (gG) {
                        p = 1.0; p *= a[j1]; p *= b[j2]; p *= c[j3]; p *= d[j4];
                        gG[j] = -e * p + reg_core * g;
                    }
                }
}

static double predict_t(const or_model *md, const or_cpos *t, const double *const *ur)
{
    if (nested(md)) return predict_nested(md, ur);
    double acc = 0.0;
    for (int64_t j = 0; j < t->K; ++j) {
        const int32_t *jj = t->pos + j * t->N;
        double p = md->G[j];
        for (int n = 0; n < md->N; ++n) p *= ur[n][jj[n]];
        acc += p;
    }
    return acc;
}

double or_predict_one(const or_model *md, const int32_t *rows)
{
    or_cpos t;
    const double *ur[OR_MAXN];
    if (!cpos_make(md, &t)) return NAN;
    entry_rows(md, rows, ur);
    double acc = predict_t(md, &t, ur);
    cpos_free(&t);
    return acc;
}

void or_predict(const or_model *md, const or_tensor *X, double *out)
{
    or_cpos t;
    int32_t rows[OR_MAXN];
    const double *ur[OR_MAXN];
    if (!cpos_make(md, &t)) return;
    for (int64_t e = 0; e < X->nnz; ++e) {
        for (int n = 0; n < md->N; ++n) rows[n] = X->idx[n * X->nnz + e];
        entry_rows(md, rows, ur);
        out[e] = predict_t(md, &t, ur);
    }
    cpos_free(&t);
}

/* ------------------------------------------------------------------ */
/* Per-entry gradients of one tensor entry, Eq (8) / Algorithm 2.
 *   e = x - x~
 *   d f / d u^(n)  = -e [G x_{-n} {u}]  + (lambda_reg / cnt_n) u^(n)
 *   d f / d G      = -e (u^(1) o ... o u^(N)) + (lambda_reg / |Omega_X|) G
 * The leave-one-out contraction w_n[k] = sum_{j : j_n = k} g_j prod_{m != n}
 * u^(m)_{i_m j_m} is formed directly (no division).
 * gU receives the N row gradients back to back (J_1 then J_2 ...); gG has
 * prod J entries.  reg_row[n] = lambda_reg / cnt_n[i_n], reg_core =
 * lambda_reg / |Omega_X|.  Returns e.                                    */

static double item_grad_t(const or_model *md, const or_cpos *t, const double *const *ur, double x,
                          const double *reg_row, double reg_core, double *gU, double *gG)
{
    const int64_t K = t->K;
    const int N = md->N;
    double xhat = predict_t(md, t, ur);
    double e = x - xhat;

    if (nested(md)) {
        loo_nested(md, ur, gU, e, reg_core, gG);
        int64_t off = 0;
        for (int n = 0; n < N; ++n) {
            double *w = gU + off;
            const double *u = ur[n];
            for (int k = 0; k < md->J[n]; ++k) w[k] = -e * w[k] + reg_row[n] * u[k];
            off += md->J[n];
        }
        return e;
    }
    int64_t off = 0;
    for (int n = 0; n < N; ++n) {
        double *w = gU + off;
        for (int k = 0; k < md->J[n]; ++k) w[k] = 0.0;
        for (int64_t j = 0; j < K; ++j) {
            const int32_t *jj = t->pos + j * N;
            double p = md->G[j];
            for (int m = 0; m < N; ++m)
                if (m != n) p *= ur[m][jj[m]];
            w[jj[n]] += p;
        }
        const double *u = ur[n];
        for (int k = 0; k < md->J[n]; ++k) w[k] = -e * w[k] + reg_row[n] * u[k];
        off += md->J[n];
    }
    for (int64_t j = 0; j < K; ++j) {
        const int32_t *jj = t->pos + j * N;
        double p = 1.0;
        for (int n = 0; n < N; ++n) p *= ur[n][jj[n]];
        gG[j] = -e * p + reg_core * md->G[j];
    }
    return e;
}

double or_tensor_item_grad(const or_model *md, const int32_t *rows, double x,
                           const double *reg_row, double reg_core,
                           double *gU, double *gG)
{
    or_cpos t;
    const double *ur[OR_MAXN];
    if (!cpos_make(md, &t)) return NAN;
    entry_rows(md, rows, ur);
    double e = item_grad_t(md, &t, ur, x, reg_row, reg_core, gU, gG);
    cpos_free(&t);
    return e;
}

/* The leave-one-out contractions w_n = G x_{-n} {u} of one entry (Eq 3 /
 * Eq 8), straight from the definition; w receives J_1 + ... + J_N values. */
static void item_w_t(const or_model *md, const or_cpos *t, const double *const *ur, double *w)
{
    if (nested(md)) {
        loo_nested(md, ur, w, 0.0, 0.0, NULL);
        return;
    }
    const int64_t K = t->K;
    const int N = md->N;
    int64_t off = 0;
    for (int n = 0; n < N; ++n) {
        for (int k = 0; k < md->J[n]; ++k) w[off + k] = 0.0;
        for (int64_t j = 0; j < K; ++j) {
            const int32_t *jj = t->pos + j * N;
            double p = md->G[j];
            for (int m = 0; m < N; ++m)
                if (m != n) p *= ur[m][jj[m]];
            w[off + jj[n]] += p;
        }
        off += md->J[n];
    }
}

void or_tensor_item_w(const or_model *md, const int32_t *rows, double *w)
{
    or_cpos t;
    const double *ur[OR_MAXN];
    if (!cpos_make(md, &t)) return;
    entry_rows(md, rows, ur);
    item_w_t(md, &t, ur, w);
    cpos_free(&t);
}

/* ------------------------------------------------------------------ */
/* The same gradients in the paper's reuse form (Definition 4, Lemma 2,
 * Definition 5, Lemma 3, Algorithm 3): S = G * (u^(1) o ... o u^(N)),
 * x~ = sum S, gradient of u^(n) from Collapse(S, n) divided elementwise by
 * u^(n), core gradient from S divided elementwise by G.  Defined only when
 * no factor entry and no core entry is zero; kept as a cross-check of the
 * direct form, not used by the epochs.  S must have prod J entries.      */

double or_tensor_item_grad_opt(const or_model *md, const int32_t *rows, double x,
                               const double *reg_row, double reg_core,
                               double *gU, double *gG, double *S)
{
    int64_t K = core_size(md);
    int32_t jj[OR_MAXN];
    double xhat = 0.0;
    for (int64_t j = 0; j < K; ++j) {
        decode(md, j, jj);
        double s = md->G[j];
        for (int n = 0; n < md->N; ++n) s *= urow(md, n, rows[n])[jj[n]];
        S[j] = s;
        xhat += s;
    }
    double e = x - xhat;
    int64_t off = 0;
    for (int n = 0; n < md->N; ++n) {
        double *w = gU + off;
        for (int k = 0; k < md->J[n]; ++k) w[k] = 0.0;
        for (int64_t j = 0; j < K; ++j) {     /* Collapse(S, n) */
            decode(md, j, jj);
            w[jj[n]] += S[j];
        }
        const double *u = urow(md, n, rows[n]);
        for (int k = 0; k < md->J[n]; ++k) w[k] = -e * (w[k] / u[k]) + reg_row[n] * u[k];
        off += md->J[n];
    }
    for (int64_t j = 0; j < K; ++j) gG[j] = -e * (S[j] / md->G[j]) + reg_core * md->G[j];
    return e;
}

/* ------------------------------------------------------------------ */
/* Per-entry gradients of one coupled-matrix entry, Eq (8) / Algorithm 1:
 *   y^ = u . v,  e = y - y^
 *   d f / d u = -lambda_m e v
 *   d f / d v = -lambda_m e u + (lambda_m lambda_reg / cntV) v          */

double or_matrix_item_grad(const double *u, const double *v, int32_t J, double y,
                           double lambda_m, double reg_v, double *gu, double *gv)
{
    double yhat = 0.0;
    for (int k = 0; k < J; ++k) yhat += u[k] * v[k];
    double e = y - yhat;
    for (int k = 0; k < J; ++k) {
        gu[k] = -lambda_m * e * v[k];
        gv[k] = -lambda_m * e * u[k] + lambda_m * reg_v * v[k];
    }
    return e;
}

/* ------------------------------------------------------------------ */
/* item helpers shared by the epochs                                   */

typedef struct {
    const or_model *md;
    const or_tensor *X;
    int32_t M;
    const or_matrix *Y;
    const or_counts *c;
    const or_hyper *h;
    int64_t off[OR_MAXM + 1];   /* first item id of each matrix */
} or_ctx;

static void ctx_init(or_ctx *cx, const or_model *md, const or_tensor *X, int32_t M,
                     const or_matrix *Y, const or_counts *c, const or_hyper *h)
{
    cx->md = md; cx->X = X; cx->M = M; cx->Y = Y; cx->c = c; cx->h = h;
    cx->off[0] = X->nnz;
    for (int m = 0; m < M; ++m) cx->off[m + 1] = cx->off[m] + Y[m].nnz;
}

/* which matrix an item id >= nX belongs to, and its local index */
static int item_matrix(const or_ctx *cx, int64_t id, int64_t *local)
{
    for (int m = 0; m < cx->M; ++m)
        if (id < cx->off[m + 1]) { *local = id - cx->off[m]; return m; }
    *local = -1;
    return -1;
}

static void tensor_rows(const or_ctx *cx, int64_t e, int32_t *rows, double *reg_row)
{
    for (int n = 0; n < cx->md->N; ++n) {
        rows[n] = cx->X->idx[n * cx->X->nnz + e];
        reg_row[n] = cx->h->lambda_reg / (double)cx->c->cnt[n][rows[n]];
    }
}

/* ------------------------------------------------------------------ */
/* One SGD epoch, Algorithm 1 with one worker: items are visited in the
 * given order; for each, all of its gradients are taken at the current
 * values and then every row it touches (and the core, for tensor entries)
 * moves by -eta times its gradient.  Returns the number of items done.   */

int64_t or_sgd_epoch(or_model *md, const or_tensor *X, int32_t M, const or_matrix *Y,
                     const or_counts *c, const or_hyper *h, const int64_t *order,
                     int64_t n_order, double eta)
{
    or_ctx cx;
    ctx_init(&cx, md, X, M, Y, c, h);
    int64_t K = core_size(md);
    int64_t R = rank_sum(md);
    double *gU = (double *)malloc(sizeof(double) * (size_t)R);
    double *gG = (double *)malloc(sizeof(double) * (size_t)K);
    double *gu = (double *)malloc(sizeof(double) * (size_t)R);
    double *gv = (double *)malloc(sizeof(double) * (size_t)R);
    int32_t rows[OR_MAXN];
    const double *ur[OR_MAXN];
    double reg_row[OR_MAXN];
    double reg_core = h->lambda_reg / (double)c->nX;
    or_cpos tab;
    if (!cpos_make(md, &tab)) { free(gU); free(gG); free(gu); free(gv); return 0; }

    for (int64_t t = 0; t < n_order; ++t) {
        int64_t id = order[t];
        if (id < X->nnz) {
            tensor_rows(&cx, id, rows, reg_row);
            entry_rows(md, rows, ur);
            item_grad_t(md, &tab, ur, X->val[id], reg_row, reg_core, gU, gG);
            int64_t off = 0;
            for (int n = 0; n < md->N; ++n) {
                double *u = md->U[n] + (int64_t)rows[n] * md->J[n];
                for (int k = 0; k < md->J[n]; ++k) u[k] -= eta * gU[off + k];
                off += md->J[n];
            }
            for (int64_t j = 0; j < K; ++j) md->G[j] -= eta * gG[j];
        } else {
            int64_t e;
            int m = item_matrix(&cx, id, &e);
            int cm = md->mode[m];
            int32_t J = md->J[cm];
            double *u = md->U[cm] + (int64_t)Y[m].row[e] * J;
            double *v = md->V[m] + (int64_t)Y[m].col[e] * J;
            double reg_v = h->lambda_reg / (double)c->cntV[m][Y[m].col[e]];
            or_matrix_item_grad(u, v, J, Y[m].val[e], h->lambda_m, reg_v, gu, gv);
            for (int k = 0; k < J; ++k) {
                u[k] -= eta * gu[k];
                v[k] -= eta * gv[k];
            }
        }
    }
    cpos_free(&tab);
    free(gU); free(gG); free(gu); free(gv);
    return n_order;
}

/* ------------------------------------------------------------------ */
/* Deterministic mini-batch epoch (this library's batched reading of the
 * per-entry SGD; with batch = 1 it is exactly or_sgd_epoch).  The order is
 * cut into consecutive batches of `batch` items; for each batch every
 * item's gradients are taken at the batch-start values, summed per
 * parameter, and each parameter moves by -eta times its sum.  Runs the
 * batches [first_batch, first_batch + n_batches) (n_batches < 0: to the
 * end).  Returns the number of batches run.
 *
 * damping != 0 selects the library's damped reading: each parameter block
 * (a factor row, a coupled-factor row, the core) also sums the curvature
 * L of its contributions -- |w_n|^2 + lambda_reg / cnt_n for a tensor
 * row, prod_n |u^(n)|^2 + lambda_reg / |Omega_X| for the core,
 * lambda_m |v|^2 for the coupled-mode row of a matrix entry and
 * lambda_m |u|^2 + lambda_m lambda_reg / cntV for its V row -- and moves
 * by -eta / max(1, (N + 1) eta L) times its gradient sum.               */

static double damped(double eta, double kappa, double L, int damping)
{
    if (!damping) return eta;
    double d = kappa * eta * L;
    return eta / (d > 1.0 ? d : 1.0);
}

int64_t or_minibatch_epoch(or_model *md, const or_tensor *X, int32_t M, const or_matrix *Y,
                           const or_counts *c, const or_hyper *h, const int64_t *order,
                           int64_t n_order, int64_t batch, double eta,
                           int64_t first_batch, int64_t n_batches, int32_t damping)
{
    or_ctx cx;
    ctx_init(&cx, md, X, M, Y, c, h);
    int N = md->N;
    int64_t K = core_size(md);
    int64_t R = rank_sum(md);
    /* gradient accumulators shaped like the parameters */
    double *aU[OR_MAXN], *aV[OR_MAXM];
    for (int n = 0; n < N; ++n) aU[n] = (double *)calloc((size_t)(md->dims[n] * md->J[n]), sizeof(double));
    for (int m = 0; m < M; ++m) aV[m] = (double *)calloc((size_t)(md->cols[m] * md->J[md->mode[m]]), sizeof(double));
    double *aG = (double *)calloc((size_t)K, sizeof(double));
    double *gU = (double *)malloc(sizeof(double) * (size_t)R);
    double *gG = (double *)malloc(sizeof(double) * (size_t)K);
    double *gu = (double *)malloc(sizeof(double) * (size_t)R);
    double *gv = (double *)malloc(sizeof(double) * (size_t)R);
    double *w = (double *)malloc(sizeof(double) * (size_t)R);
    double *LU[OR_MAXN], *LV[OR_MAXM];
    for (int n = 0; n < N; ++n) LU[n] = (double *)calloc((size_t)md->dims[n], sizeof(double));
    for (int m = 0; m < M; ++m) LV[m] = (double *)calloc((size_t)md->cols[m], sizeof(double));
    double LG = 0.0;
    double kappa = (double)(N + 1);
    int32_t rows[OR_MAXN];
    const double *ur[OR_MAXN];
    double reg_row[OR_MAXN];
    double reg_core = h->lambda_reg / (double)c->nX;
    or_cpos tab;
    if (!cpos_make(md, &tab)) return -1;

    int64_t nb_total = (n_order + batch - 1) / batch;
    int64_t last = n_batches < 0 ? nb_total : first_batch + n_batches;
    if (last > nb_total) last = nb_total;
    int64_t done = 0;
    for (int64_t b = first_batch; b < last; ++b) {
        int64_t t0 = b * batch, t1 = t0 + batch;
        if (t1 > n_order) t1 = n_order;
        /* 1: gradients at the batch-start values, summed per parameter */
        for (int64_t t = t0; t < t1; ++t) {
            int64_t id = order[t];
            if (id < X->nnz) {
                tensor_rows(&cx, id, rows, reg_row);
                entry_rows(md, rows, ur);
                item_grad_t(md, &tab, ur, X->val[id], reg_row, reg_core, gU, gG);
                int64_t off = 0;
                for (int n = 0; n < N; ++n) {
                    double *a = aU[n] + (int64_t)rows[n] * md->J[n];
                    for (int k = 0; k < md->J[n]; ++k) a[k] += gU[off + k];
                    off += md->J[n];
                }
                for (int64_t j = 0; j < K; ++j) aG[j] += gG[j];
                if (damping) {
                    item_w_t(md, &tab, ur, w);
                    double pu = 1.0;
                    off = 0;
                    for (int n = 0; n < N; ++n) {
                        const double *u = urow(md, n, rows[n]);
                        double ww = 0.0, uu = 0.0;
                        for (int k = 0; k < md->J[n]; ++k) { ww += w[off + k] * w[off + k]; uu += u[k] * u[k]; }
                        LU[n][rows[n]] += ww + reg_row[n];
                        pu *= uu;
                        off += md->J[n];
                    }
                    if (md->cp) {
                        /* ||d x~ / d g||^2 over the diagonal only */
                        pu = 0.0;
                        for (int r = 0; r < md->J[0]; ++r) {
                            double q = 1.0;
                            for (int n = 0; n < N; ++n) {
                                double v = urow(md, n, rows[n])[r];
                                q *= v * v;
                            }
                            pu += q;
                        }
                    }
                    LG += pu + reg_core;
                }
            } else {
                int64_t e;
                int m = item_matrix(&cx, id, &e);
                int cm = md->mode[m];
                int32_t J = md->J[cm];
                const double *u = md->U[cm] + (int64_t)Y[m].row[e] * J;
                const double *v = md->V[m] + (int64_t)Y[m].col[e] * J;
                double reg_v = h->lambda_reg / (double)c->cntV[m][Y[m].col[e]];
                or_matrix_item_grad(u, v, J, Y[m].val[e], h->lambda_m, reg_v, gu, gv);
                double *au = aU[cm] + (int64_t)Y[m].row[e] * J;
                double *av = aV[m] + (int64_t)Y[m].col[e] * J;
                for (int k = 0; k < J; ++k) { au[k] += gu[k]; av[k] += gv[k]; }
                if (damping) {
                    double uu = 0.0, vv = 0.0;
                    for (int k = 0; k < J; ++k) { uu += u[k] * u[k]; vv += v[k] * v[k]; }
                    LU[cm][Y[m].row[e]] += h->lambda_m * vv;
                    LV[m][Y[m].col[e]] += h->lambda_m * uu + h->lambda_m * reg_v;
                }
            }
        }
        /* 2: apply and clear the touched accumulators */
        for (int64_t t = t0; t < t1; ++t) {
            int64_t id = order[t];
            if (id < X->nnz) {
                for (int n = 0; n < N; ++n) {
                    int64_t i = X->idx[n * X->nnz + id];
                    double *u = md->U[n] + i * md->J[n];
                    double *a = aU[n] + i * md->J[n];
                    double st = damped(eta, kappa, LU[n][i], damping);
                    for (int k = 0; k < md->J[n]; ++k) { u[k] -= st * a[k]; a[k] = 0.0; }
                    LU[n][i] = 0.0;
                }
            } else {
                int64_t e;
                int m = item_matrix(&cx, id, &e);
                int cm = md->mode[m];
                int32_t J = md->J[cm];
                double *u = md->U[cm] + (int64_t)Y[m].row[e] * J;
                double *au = aU[cm] + (int64_t)Y[m].row[e] * J;
                double *v = md->V[m] + (int64_t)Y[m].col[e] * J;
                double *av = aV[m] + (int64_t)Y[m].col[e] * J;
                double su = damped(eta, kappa, LU[cm][Y[m].row[e]], damping);
                double sv = damped(eta, kappa, LV[m][Y[m].col[e]], damping);
                for (int k = 0; k < J; ++k) {
                    u[k] -= su * au[k]; au[k] = 0.0;
                    v[k] -= sv * av[k]; av[k] = 0.0;
                }
                LU[cm][Y[m].row[e]] = 0.0;
                LV[m][Y[m].col[e]] = 0.0;
            }
        }
        double sg = damped(eta, kappa, LG, damping);
        for (int64_t j = 0; j < K; ++j) { md->G[j] -= sg * aG[j]; aG[j] = 0.0; }
        LG = 0.0;
        ++done;
    }
    for (int n = 0; n < N; ++n) { free(aU[n]); free(LU[n]); }
    for (int m = 0; m < M; ++m) { free(aV[m]); free(LV[m]); }
    cpos_free(&tab);
    free(aG); free(gU); free(gG); free(gu); free(gv); free(w);
    return done;
}

/* ------------------------------------------------------------------ */
/* The same deterministic mini-batch epoch with `threads` worker threads,
 * giving bitwise the results of or_minibatch_epoch.  Per batch, in blocks
 * of at most OR_MT_BLOCK items:
 *   1. the threads take contiguous ranges of items and evaluate each item's
 *      error, row gradients and curvature terms at the batch-start values
 *      (the same expressions as above), into per-item slots;
 *   2. one thread adds the slots to the row accumulators in item order;
 *   3. the threads take ranges of core values j and add, item by item in
 *      order, the item's core-gradient term -e prod_n u^(n) + reg G_j.
 * Every accumulator therefore sums the same terms in the same order as the
 * sequential loop; only the evaluation is spread over threads.  The apply
 * step is the sequential one.                                            */

#define OR_MT_BLOCK 16384

typedef struct {
    const or_ctx *cx;
    const or_cpos *tab;
    const int64_t *order;
    int64_t t0, n;            /* block: items order[t0 .. t0 + n) */
    int32_t damping;
    double reg_core;
    int64_t R;                /* sum of ranks: slot width */
    double *e;                /* [n]      tensor error; unused for matrices */
    double *g;                /* [n][2R]  row gradients (tensor: J_1..J_N;
                                            matrix: g_u then g_v)          */
    double *cu;               /* [n][N]   curvature terms per row        */
    double *cg;               /* [n]      core curvature term            */
    int32_t *rows;            /* [n][N]   tensor rows                    */
    /* phase 3 */
    double *aG;
    int64_t j0, j1;
    int64_t lo, hi;           /* phase 1: item range of this thread */
} or_mt_job;

static void mt_eval(or_mt_job *jb)
{
    const or_ctx *cx = jb->cx;
    const or_model *md = cx->md;
    const int N = md->N;
    const int64_t R = jb->R;
    double *w = (double *)malloc(sizeof(double) * (size_t)R);
    double *gG = (double *)malloc(sizeof(double) * (size_t)jb->tab->K);
    double reg_row[OR_MAXN];
    const double *ur[OR_MAXN];
    for (int64_t i = jb->lo; i < jb->hi; ++i) {
        int64_t id = jb->order[jb->t0 + i];
        double *g = jb->g + i * 2 * R;
        if (id < cx->X->nnz) {
            int32_t *rows = jb->rows + i * N;
            tensor_rows(cx, id, rows, reg_row);
            entry_rows(md, rows, ur);
            jb->e[i] = item_grad_t(md, jb->tab, ur, cx->X->val[id], reg_row, jb->reg_core, g, gG);
            if (jb->damping) {
                item_w_t(md, jb->tab, ur, w);
                double pu = 1.0;
                int64_t off = 0;
                for (int n = 0; n < N; ++n) {
                    const double *u = ur[n];
                    double ww = 0.0, uu = 0.0;
                    for (int k = 0; k < md->J[n]; ++k) { ww += w[off + k] * w[off + k]; uu += u[k] * u[k]; }
                    jb->cu[i * N + n] = ww + reg_row[n];
                    pu *= uu;
                    off += md->J[n];
                }
                if (md->cp) {
                    pu = 0.0;
                    for (int r = 0; r < md->J[0]; ++r) {
                        double q = 1.0;
                        for (int n = 0; n < N; ++n) {
                            double v = ur[n][r];
                            q *= v * v;
                        }
                        pu += q;
                    }
                }
                jb->cg[i] = pu + jb->reg_core;
            }
        } else {
            int64_t e;
            int m = item_matrix(cx, id, &e);
            int cm = md->mode[m];
            int32_t J = md->J[cm];
            const double *u = md->U[cm] + (int64_t)cx->Y[m].row[e] * J;
            const double *v = md->V[m] + (int64_t)cx->Y[m].col[e] * J;
            double reg_v = cx->h->lambda_reg / (double)cx->c->cntV[m][cx->Y[m].col[e]];
            or_matrix_item_grad(u, v, J, cx->Y[m].val[e], cx->h->lambda_m, reg_v, g, g + J);
            if (jb->damping) {
                double uu = 0.0, vv = 0.0;
                for (int k = 0; k < J; ++k) { uu += u[k] * u[k]; vv += v[k] * v[k]; }
                jb->cu[i * N + 0] = cx->h->lambda_m * vv;
                jb->cu[i * N + 1] = cx->h->lambda_m * uu + cx->h->lambda_m * reg_v;
            }
        }
    }
    free(w);
    free(gG);
}

static void *mt_eval_thread(void *arg)
{
    mt_eval((or_mt_job *)arg);
    return NULL;
}

/* core-gradient terms of the block's tensor items, core values [j0, j1) */
static void *mt_core_thread(void *arg)
{
    or_mt_job *jb = (or_mt_job *)arg;
    const or_ctx *cx = jb->cx;
    const or_model *md = cx->md;
    const int N = md->N;
    const double *ur[OR_MAXN];
    for (int64_t i = 0; i < jb->n; ++i) {
        int64_t id = jb->order[jb->t0 + i];
        if (id >= cx->X->nnz) continue;
        entry_rows(md, jb->rows + i * N, ur);
        const double e = jb->e[i];
        for (int64_t j = jb->j0; j < jb->j1; ++j) {
            const int32_t *jj = jb->tab->pos + j * N;
            double p = 1.0;
            for (int n = 0; n < N; ++n) p *= ur[n][jj[n]];
            jb->aG[j] += -e * p + jb->reg_core * md->G[j];
        }
    }
    return NULL;
}

static void mt_run(void *(*fn)(void *), or_mt_job *jobs, int threads)
{
    pthread_t th[64];
    for (int k = 1; k < threads; ++k) pthread_create(&th[k], NULL, fn, &jobs[k]);
    fn(&jobs[0]);
    for (int k = 1; k < threads; ++k) pthread_join(th[k], NULL);
}

int64_t or_minibatch_epoch_mt(or_model *md, const or_tensor *X, int32_t M, const or_matrix *Y,
                              const or_counts *c, const or_hyper *h, const int64_t *order,
                              int64_t n_order, int64_t batch, double eta,
                              int64_t first_batch, int64_t n_batches, int32_t damping,
                              int32_t threads)
{
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    or_ctx cx;
    ctx_init(&cx, md, X, M, Y, c, h);
    const int N = md->N;
    const int64_t K = core_size(md);
    const int64_t R = rank_sum(md);
    or_cpos tab;
    if (!cpos_make(md, &tab)) return -1;
    double *aU[OR_MAXN], *aV[OR_MAXM], *LU[OR_MAXN], *LV[OR_MAXM];
    for (int n = 0; n < N; ++n) aU[n] = (double *)calloc((size_t)(md->dims[n] * md->J[n]), sizeof(double));
    for (int m = 0; m < M; ++m) aV[m] = (double *)calloc((size_t)(md->cols[m] * md->J[md->mode[m]]), sizeof(double));
    for (int n = 0; n < N; ++n) LU[n] = (double *)calloc((size_t)md->dims[n], sizeof(double));
    for (int m = 0; m < M; ++m) LV[m] = (double *)calloc((size_t)md->cols[m], sizeof(double));
    double *aG = (double *)calloc((size_t)K, sizeof(double));
    double LG = 0.0;
    const double kappa = (double)(N + 1);
    const double reg_core = h->lambda_reg / (double)c->nX;
    const int64_t S = OR_MT_BLOCK;
    double *be = (double *)malloc(sizeof(double) * (size_t)S);
    double *bg = (double *)malloc(sizeof(double) * (size_t)(S * 2 * R));
    double *bcu = (double *)malloc(sizeof(double) * (size_t)(S * N));
    double *bcg = (double *)malloc(sizeof(double) * (size_t)S);
    int32_t *brows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S * N));
    or_mt_job jobs[64];

    int64_t nb_total = (n_order + batch - 1) / batch;
    int64_t last = n_batches < 0 ? nb_total : first_batch + n_batches;
    if (last > nb_total) last = nb_total;
    int64_t done = 0;
    for (int64_t b = first_batch; b < last; ++b) {
        int64_t t0 = b * batch, t1 = t0 + batch;
        if (t1 > n_order) t1 = n_order;
        for (int64_t s0 = t0; s0 < t1; s0 += S) {
            const int64_t n = (t1 - s0 < S) ? t1 - s0 : S;
            for (int k = 0; k < threads; ++k) {
                or_mt_job *jb = &jobs[k];
                jb->cx = &cx; jb->tab = &tab; jb->order = order; jb->t0 = s0; jb->n = n;
                jb->damping = damping; jb->reg_core = reg_core; jb->R = R;
                jb->e = be; jb->g = bg; jb->cu = bcu; jb->cg = bcg; jb->rows = brows; jb->aG = aG;
                jb->lo = n * k / threads; jb->hi = n * (k + 1) / threads;
                jb->j0 = K * k / threads; jb->j1 = K * (k + 1) / threads;
            }
            /* 1: evaluation */
            mt_run(mt_eval_thread, jobs, threads);
            /* 2: row sums in item order */
            for (int64_t i = 0; i < n; ++i) {
                int64_t id = order[s0 + i];
                const double *g = bg + i * 2 * R;
                if (id < X->nnz) {
                    const int32_t *rows = brows + i * N;
                    int64_t off = 0;
                    for (int q = 0; q < N; ++q) {
                        double *a = aU[q] + (int64_t)rows[q] * md->J[q];
                        for (int k = 0; k < md->J[q]; ++k) a[k] += g[off + k];
                        off += md->J[q];
                    }
                    if (damping) {
                        for (int q = 0; q < N; ++q) LU[q][rows[q]] += bcu[i * N + q];
                        LG += bcg[i];
                    }
                } else {
                    int64_t e;
                    int m = item_matrix(&cx, id, &e);
                    int cm = md->mode[m];
                    int32_t J = md->J[cm];
                    double *au = aU[cm] + (int64_t)Y[m].row[e] * J;
                    double *av = aV[m] + (int64_t)Y[m].col[e] * J;
                    for (int k = 0; k < J; ++k) { au[k] += g[k]; av[k] += g[J + k]; }
                    if (damping) {
                        LU[cm][Y[m].row[e]] += bcu[i * N + 0];
                        LV[m][Y[m].col[e]] += bcu[i * N + 1];
                    }
                }
            }
            /* 3: core-gradient sums, by ranges of core values */
            mt_run(mt_core_thread, jobs, threads);
        }
        /* apply and clear the touched accumulators (as in the sequential epoch) */
        for (int64_t t = t0; t < t1; ++t) {
            int64_t id = order[t];
            if (id < X->nnz) {
                for (int n = 0; n < N; ++n) {
                    int64_t i = X->idx[n * X->nnz + id];
                    double *u = md->U[n] + i * md->J[n];
                    double *a = aU[n] + i * md->J[n];
                    double st = damped(eta, kappa, LU[n][i], damping);
                    for (int k = 0; k < md->J[n]; ++k) { u[k] -= st * a[k]; a[k] = 0.0; }
                    LU[n][i] = 0.0;
                }
            } else {
                int64_t e;
                int m = item_matrix(&cx, id, &e);
                int cm = md->mode[m];
                int32_t J = md->J[cm];
                double *u = md->U[cm] + (int64_t)Y[m].row[e] * J;
                double *au = aU[cm] + (int64_t)Y[m].row[e] * J;
                double *v = md->V[m] + (int64_t)Y[m].col[e] * J;
                double *av = aV[m] + (int64_t)Y[m].col[e] * J;
                double su = damped(eta, kappa, LU[cm][Y[m].row[e]], damping);
                double sv = damped(eta, kappa, LV[m][Y[m].col[e]], damping);
                for (int k = 0; k < J; ++k) {
                    u[k] -= su * au[k]; au[k] = 0.0;
                    v[k] -= sv * av[k]; av[k] = 0.0;
                }
                LU[cm][Y[m].row[e]] = 0.0;
                LV[m][Y[m].col[e]] = 0.0;
            }
        }
        double sg = damped(eta, kappa, LG, damping);
        for (int64_t j = 0; j < K; ++j) { md->G[j] -= sg * aG[j]; aG[j] = 0.0; }
        LG = 0.0;
        ++done;
    }
    for (int n = 0; n < N; ++n) { free(aU[n]); free(LU[n]); }
    for (int m = 0; m < M; ++m) { free(aV[m]); free(LV[m]); }
    free(aG); free(be); free(bg); free(bcu); free(bcg); free(brows);
    cpos_free(&tab);
    return done;
}

/* ------------------------------------------------------------------ */
/* Objective f of Eq (7), in the per-entry form summed over all items:
 *   f_t = sum_alpha e^2 + lambda_reg ||G||^2 + lambda_reg sum_n sum_{i: cnt>0} ||u_i||^2
 *   f_m = sum_m [ sum_beta e^2 + lambda_reg sum_{k: cntV>0} ||v_k||^2 ]
 *   f   = f_t / 2 + lambda_m f_m / 2
 * out[0] = f, out[1] = f_t, out[2] = f_m.                                */

void or_loss(const or_model *md, const or_tensor *X, int32_t M, const or_matrix *Y,
             const or_counts *c, const or_hyper *h, double *out)
{
    int32_t rows[OR_MAXN];
    const double *ur[OR_MAXN];
    double sse = 0.0;
    or_cpos tab;
    if (!cpos_make(md, &tab)) { out[0] = out[1] = out[2] = NAN; return; }
    for (int64_t e = 0; e < X->nnz; ++e) {
        for (int n = 0; n < md->N; ++n) rows[n] = X->idx[n * X->nnz + e];
        entry_rows(md, rows, ur);
        double r = X->val[e] - predict_t(md, &tab, ur);
        sse += r * r;
    }
    cpos_free(&tab);
    double reg = 0.0;
    int64_t K = core_size(md);
    for (int64_t j = 0; j < K; ++j) reg += md->G[j] * md->G[j];
    for (int n = 0; n < md->N; ++n)
        for (int64_t i = 0; i < md->dims[n]; ++i) {
            if (c->cnt[n][i] == 0) continue;
            const double *u = urow(md, n, i);
            for (int k = 0; k < md->J[n]; ++k) reg += u[k] * u[k];
        }
    double ft = sse + h->lambda_reg * reg;
    double fm = 0.0;
    for (int m = 0; m < M; ++m) {
        int cm = md->mode[m];
        int32_t J = md->J[cm];
        double s = 0.0;
        for (int64_t e = 0; e < Y[m].nnz; ++e) {
            const double *u = md->U[cm] + (int64_t)Y[m].row[e] * J;
            const double *v = md->V[m] + (int64_t)Y[m].col[e] * J;
            double yh = 0.0;
            for (int k = 0; k < J; ++k) yh += u[k] * v[k];
            double r = Y[m].val[e] - yh;
            s += r * r;
        }
        double rv = 0.0;
        for (int64_t k = 0; k < md->cols[m]; ++k) {
            if (c->cntV[m][k] == 0) continue;
            const double *v = md->V[m] + k * J;
            for (int q = 0; q < J; ++q) rv += v[q] * v[q];
        }
        fm += s + h->lambda_reg * rv;
    }
    out[0] = 0.5 * ft + 0.5 * h->lambda_m * fm;
    out[1] = ft;
    out[2] = fm;
}

/* Held-out RMSE (Section 4.1, "Measure"): sqrt(mean over the test
 * entries of (x - x~)^2).                                               */
double or_rmse(const or_model *md, const or_tensor *T)
{
    if (T->nnz == 0) return 0.0;
    int32_t rows[OR_MAXN];
    const double *ur[OR_MAXN];
    double s = 0.0;
    or_cpos tab;
    if (!cpos_make(md, &tab)) return NAN;
    for (int64_t e = 0; e < T->nnz; ++e) {
        for (int n = 0; n < md->N; ++n) rows[n] = T->idx[n * T->nnz + e];
        entry_rows(md, rows, ur);
        double r = T->val[e] - predict_t(md, &tab, ur);
        s += r * r;
    }
    cpos_free(&tab);
    return sqrt(s / (double)T->nnz);
}

/* ------------------------------------------------------------------ */
/* Full gradient of f: the sum over all items of their per-entry
 * gradients (Eq 8).  Outputs are shaped like the parameters and are
 * overwritten.                                                           */

void or_full_grad(const or_model *md, const or_tensor *X, int32_t M, const or_matrix *Y,
                  const or_counts *c, const or_hyper *h,
                  double **dU, double *dG, double **dV)
{
    or_ctx cx;
    ctx_init(&cx, md, X, M, Y, c, h);
    int N = md->N;
    int64_t K = core_size(md);
    int64_t R = rank_sum(md);
    for (int n = 0; n < N; ++n) memset(dU[n], 0, sizeof(double) * (size_t)(md->dims[n] * md->J[n]));
    for (int m = 0; m < M; ++m) memset(dV[m], 0, sizeof(double) * (size_t)(md->cols[m] * md->J[md->mode[m]]));
    memset(dG, 0, sizeof(double) * (size_t)K);
    double *gU = (double *)malloc(sizeof(double) * (size_t)R);
    double *gG = (double *)malloc(sizeof(double) * (size_t)K);
    double *gu = (double *)malloc(sizeof(double) * (size_t)R);
    double *gv = (double *)malloc(sizeof(double) * (size_t)R);
    int32_t rows[OR_MAXN];
    const double *ur[OR_MAXN];
    double reg_row[OR_MAXN];
    double reg_core = h->lambda_reg / (double)c->nX;
    or_cpos tab;
    if (!cpos_make(md, &tab)) { free(gU); free(gG); free(gu); free(gv); return; }
    for (int64_t e = 0; e < X->nnz; ++e) {
        tensor_rows(&cx, e, rows, reg_row);
        entry_rows(md, rows, ur);
        item_grad_t(md, &tab, ur, X->val[e], reg_row, reg_core, gU, gG);
        int64_t off = 0;
        for (int n = 0; n < N; ++n) {
            double *a = dU[n] + (int64_t)rows[n] * md->J[n];
            for (int k = 0; k < md->J[n]; ++k) a[k] += gU[off + k];
            off += md->J[n];
        }
        for (int64_t j = 0; j < K; ++j) dG[j] += gG[j];
    }
    for (int m = 0; m < M; ++m) {
        int cm = md->mode[m];
        int32_t J = md->J[cm];
        for (int64_t e = 0; e < Y[m].nnz; ++e) {
            const double *u = md->U[cm] + (int64_t)Y[m].row[e] * J;
            const double *v = md->V[m] + (int64_t)Y[m].col[e] * J;
            double reg_v = h->lambda_reg / (double)c->cntV[m][Y[m].col[e]];
            or_matrix_item_grad(u, v, J, Y[m].val[e], h->lambda_m, reg_v, gu, gv);
            double *au = dU[cm] + (int64_t)Y[m].row[e] * J;
            double *av = dV[m] + (int64_t)Y[m].col[e] * J;
            for (int k = 0; k < J; ++k) { au[k] += gu[k]; av[k] += gv[k]; }
        }
    }
    cpos_free(&tab);
    free(gU); free(gG); free(gu); free(gv);
}

/* ------------------------------------------------------------------ */
/* Adjoint of the prediction map.  Forward: x~_e = G x {u}_e for every
 * tensor entry (Eq 4) and y^_e = u^(c)_r . v_k for every entry of each
 * coupled matrix.  Given upstream sensitivities gx[e] = dL/dx~_e and
 * gy[m][e] = dL/dy^_e, return dL/dU, dL/dG, dL/dV:
 *   dL/du^(n)_{i_n} += gx[e] [G x_{-n} {u}_e]       (same contraction as Eq 8)
 *   dL/dG          += gx[e] (u^(1) o ... o u^(N))
 *   dL/du^(c)_r    += gy[e] v_k ,  dL/dv_k += gy[e] u^(c)_r
 * Outputs overwritten.                                                    */

void or_adjoint(const or_model *md, const or_tensor *X, const double *gx,
                int32_t M, const or_matrix *Y, const double *const *gy,
                double **dU, double *dG, double **dV)
{
    int N = md->N;
    int64_t K = core_size(md);
    int32_t jj[OR_MAXN];
    int32_t rows[OR_MAXN];
    for (int n = 0; n < N; ++n) memset(dU[n], 0, sizeof(double) * (size_t)(md->dims[n] * md->J[n]));
    for (int m = 0; m < M; ++m) memset(dV[m], 0, sizeof(double) * (size_t)(md->cols[m] * md->J[md->mode[m]]));
    memset(dG, 0, sizeof(double) * (size_t)K);
    for (int64_t e = 0; e < X->nnz; ++e) {
        for (int n = 0; n < N; ++n) rows[n] = X->idx[n * X->nnz + e];
        for (int64_t j = 0; j < K; ++j) {
            decode(md, j, jj);
            double p = 1.0;
            for (int n = 0; n < N; ++n) p *= urow(md, n, rows[n])[jj[n]];
            dG[j] += gx[e] * p;
            for (int n = 0; n < N; ++n) {
                double q = md->G[j];
                for (int m = 0; m < N; ++m)
                    if (m != n) q *= urow(md, m, rows[m])[jj[m]];
                dU[n][(int64_t)rows[n] * md->J[n] + jj[n]] += gx[e] * q;
            }
        }
    }
    for (int m = 0; m < M; ++m) {
        int cm = md->mode[m];
        int32_t J = md->J[cm];
        for (int64_t e = 0; e < Y[m].nnz; ++e) {
            int64_t r = Y[m].row[e], k = Y[m].col[e];
            for (int q = 0; q < J; ++q) {
                dU[cm][r * J + q] += gy[m][e] * md->V[m][k * J + q];
                dV[m][k * J + q] += gy[m][e] * md->U[cm][r * J + q];
            }
        }
    }
}

/* coupled-matrix predictions y^_e = u^(c)_r . v_k */
void or_matrix_predict(const or_model *md, int32_t m, const or_matrix *Y, double *out)
{
    int cm = md->mode[m];
    int32_t J = md->J[cm];
    for (int64_t e = 0; e < Y->nnz; ++e) {
        const double *u = md->U[cm] + (int64_t)Y->row[e] * J;
        const double *v = md->V[m] + (int64_t)Y->col[e] * J;
        double s = 0.0;
        for (int q = 0; q < J; ++q) s += u[q] * v[q];
        out[e] = s;
    }
}
