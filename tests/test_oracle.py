"""Pins for the FP64 oracle (CPU only).

Each test ties an oracle routine to something other than itself: the dense
Kronecker form of the Tucker model, finite differences, closed forms at
special points, the paper's equivalence lemmas, or brute force on tiny
inputs.  A plausible slip in the oracle (a dropped term, a wrong sign or
index, a transposed operand, a missing 1/|Omega| factor) fails one of them.
"""
import numpy as np
import pytest

import oracle
from synth import get_config, make_problem, init_params, item_order
from tests.dense_ref import damped_batch_step, dense_predict, dense_tucker, fd_grad, item_phi, rel


def _problem(name, **kw):
    cfg = get_config(name, **kw)
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    params = oracle.Params.from_arrays(U, G, V, [s.mode for s in cfg.matrices])
    return cfg, p, params


def _rand_params(rng, dims, ranks, mats, scale=0.7):
    U = [rng.normal(0, scale, size=(I, J)) for I, J in zip(dims, ranks)]
    G = rng.normal(0, scale, size=tuple(ranks))
    V = [rng.normal(0, scale, size=(K, ranks[c])) for (c, K) in mats]
    return oracle.Params.from_arrays(U, G, V, [c for c, _ in mats])


# ---------------------------------------------------------------- Eq (4)

@pytest.mark.parametrize("name", ["tiny3", "tiny4"])
def test_predict_matches_dense_kronecker(name):
    cfg, p, _ = _problem(name)
    rng = np.random.default_rng(0)
    params = _rand_params(rng, cfg.dims, cfg.ranks, [(s.mode, s.cols) for s in cfg.matrices])
    # every coordinate of the (tiny) tensor, not just the observed ones
    grid = np.stack(np.meshgrid(*[np.arange(I) for I in cfg.dims], indexing="ij")).reshape(cfg.order, -1)
    got = oracle.predict(params, grid)
    want = dense_predict(params.U, params.G, grid)
    assert rel(got, want) < 1e-13


def test_predict_rank_one_core():
    rng = np.random.default_rng(1)
    params = _rand_params(rng, (5, 4, 3), (1, 1, 1), [])
    idx = np.array([[0, 4, 2], [3, 1, 0], [2, 2, 1]])
    got = oracle.predict(params, idx)
    g = params.G.item()
    want = [g * params.U[0][i, 0] * params.U[1][j, 0] * params.U[2][k, 0] for i, j, k in idx.T]
    assert rel(got, want) < 1e-14


def test_predict_hyperdiagonal_core_is_cp():
    # a hyper-diagonal core turns the Tucker model into CP (Section 2.2)
    rng = np.random.default_rng(2)
    R = 3
    params = _rand_params(rng, (6, 5, 4), (R, R, R), [])
    lam = rng.normal(size=R)
    G = np.zeros((R, R, R))
    for r in range(R):
        G[r, r, r] = lam[r]
    params.G[...] = G
    idx = np.array([[0, 5, 3, 2], [4, 0, 1, 1], [3, 2, 0, 1]])
    got = oracle.predict(params, idx)
    want = [np.sum(lam * params.U[0][i] * params.U[1][j] * params.U[2][k]) for i, j, k in idx.T]
    assert rel(got, want) < 1e-14


def test_two_mode_identity_core_is_matrix_factorisation():
    rng = np.random.default_rng(3)
    params = _rand_params(rng, (7, 6), (3, 3), [])
    params.G[...] = np.eye(3)
    idx = np.array([[0, 1, 6], [5, 2, 0]])
    got = oracle.predict(params, idx)
    want = [params.U[0][i] @ params.U[1][j] for i, j in idx.T]
    assert rel(got, want) < 1e-14


# ---------------------------------------------------------------- Eq (8)

@pytest.mark.parametrize("dims,ranks", [((4, 3, 5), (2, 3, 2)), ((3, 2, 2, 3), (2, 2, 1, 2))])
def test_tensor_item_grad_matches_finite_differences(dims, ranks):
    rng = np.random.default_rng(4)
    params = _rand_params(rng, dims, ranks, [])
    rows = [int(rng.integers(0, I)) for I in dims]
    x = 3.0
    reg_row = rng.uniform(0.05, 0.5, size=len(dims))
    reg_core = 0.03
    e, gU, gG = oracle.tensor_item_grad(params, rows, x, reg_row, reg_core)
    assert abs(e - (x - dense_predict(params.U, params.G, np.array(rows)[:, None])[0])) < 1e-13

    def phi():
        return item_phi(params.U, params.G, rows, x, reg_row, reg_core)

    for n in range(len(dims)):
        mask = np.zeros_like(params.U[n], dtype=bool)
        mask[rows[n]] = True
        fd = fd_grad(phi, params.U[n], mask=mask)[rows[n]]
        assert rel(gU[n], fd) < 1e-7, n
    assert rel(gG, fd_grad(phi, params.G)) < 1e-7


def test_opt_form_equals_direct_form():
    # Lemma 2 (x~ = sum of S) and Lemma 3 (Collapse / elementwise-division form
    # equals Eq 8) on inputs with no zero entries.
    rng = np.random.default_rng(5)
    for dims, ranks in [((4, 3, 5), (2, 3, 2)), ((3, 4, 2, 3), (2, 3, 2, 2)), ((6, 5, 4), (4, 3, 5))]:
        params = _rand_params(rng, dims, ranks, [])
        for u in params.U:
            u[np.abs(u) < 1e-3] = 0.5
        params.G[np.abs(params.G) < 1e-3] = 0.5
        rows = [int(rng.integers(0, I)) for I in dims]
        reg_row = rng.uniform(0.05, 0.5, size=len(dims))
        e1, gU1, gG1 = oracle.tensor_item_grad(params, rows, 2.0, reg_row, 0.01)
        e2, gU2, gG2, S = oracle.tensor_item_grad_opt(params, rows, 2.0, reg_row, 0.01)
        xhat = dense_predict(params.U, params.G, np.array(rows)[:, None])[0]
        assert abs(S.sum() - xhat) < 1e-12 * max(1, abs(xhat))
        assert abs(e1 - e2) < 1e-12
        for a, b in zip(gU1, gU2):
            assert rel(a, b) < 1e-11
        assert rel(gG1, gG2) < 1e-11


def test_matrix_item_grad_matches_finite_differences():
    rng = np.random.default_rng(6)
    u, v = rng.normal(size=4), rng.normal(size=4)
    y, lam_m, reg_v = 0.7, 10.0, 0.2
    e, gu, gv = oracle.matrix_item_grad(u, v, y, lam_m, reg_v)
    assert abs(e - (y - u @ v)) < 1e-14

    def phi():
        r = y - u @ v
        return 0.5 * lam_m * (r * r + reg_v * (v @ v))

    assert rel(gu, fd_grad(phi, u)) < 1e-8
    assert rel(gv, fd_grad(phi, v)) < 1e-8


# ---------------------------------------------------------------- Eq (7)

def test_loss_of_zero_model_is_half_sum_of_squares():
    cfg, p, params = _problem("tiny4")
    for a in params.U + [params.G] + params.V:
        a[...] = 0.0
    f, ft, fm = oracle.loss(params, p)
    want_t = np.sum(p.train_val ** 2)
    want_m = sum(np.sum(v ** 2) for v in p.mat_val)
    assert abs(ft - want_t) < 1e-12 * want_t
    assert abs(fm - want_m) < 1e-12 * max(want_m, 1)
    assert abs(f - (0.5 * want_t + 0.5 * cfg.lambda_m * want_m)) < 1e-12 * f


def test_loss_gradient_matches_full_gradient():
    # the oracle's f must be consistent with the sum of its per-entry gradients
    cfg, p, _ = _problem("tiny3")
    rng = np.random.default_rng(7)
    params = _rand_params(rng, cfg.dims, cfg.ranks, [(s.mode, s.cols) for s in cfg.matrices], 0.5)
    dU, dG, dV = oracle.full_grad(params, p)

    def f():
        return oracle.loss(params, p)[0]

    for n in range(cfg.order):
        assert rel(dU[n], fd_grad(f, params.U[n])) < 1e-7
    assert rel(dG, fd_grad(f, params.G)) < 1e-7
    for m in range(len(params.V)):
        assert rel(dV[m], fd_grad(f, params.V[m])) < 1e-7


def test_loss_regularises_only_observed_rows():
    cfg, p, params = _problem("tiny3", matrices=(), nnz=12, dims=(10, 8, 9))
    cnt, cntV = oracle.counts(params, p)
    f0 = oracle.loss(params, p)[0]
    # rows never observed in training carry no regularisation: moving them
    # changes nothing; moving an observed row does change f
    unseen = [np.flatnonzero(c == 0) for c in cnt]
    for n, rows in enumerate(unseen):
        params.U[n][rows] += 3.0
    assert any(len(r) for r in unseen)
    assert abs(oracle.loss(params, p)[0] - f0) < 1e-12 * f0
    seen = np.flatnonzero(cnt[0] > 0)[0]
    params.U[0][seen] += 0.1
    assert abs(oracle.loss(params, p)[0] - f0) > 1e-6


def test_counts_are_histograms():
    cfg, p, params = _problem("cfg1")
    cnt, cntV = oracle.counts(params, p)
    for n in range(cfg.order):
        assert np.array_equal(cnt[n], np.bincount(p.train_idx[n], minlength=cfg.dims[n]))
    assert np.array_equal(cntV[0], np.bincount(p.mat_col[0], minlength=cfg.matrices[0].cols))


# ---------------------------------------------------------------- RMSE

def test_rmse_zero_model_and_dense_model():
    cfg, p, params = _problem("tiny4")
    r_model = oracle.rmse(params, p.test_idx, p.test_val)
    want = np.sqrt(np.mean((p.test_val - dense_predict(params.U, params.G, p.test_idx)) ** 2))
    assert abs(r_model - want) < 1e-13
    for a in params.U + [params.G]:
        a[...] = 0.0
    assert abs(oracle.rmse(params, p.test_idx, p.test_val) - np.sqrt(np.mean(p.test_val ** 2))) < 1e-13


# ---------------------------------------------------------------- epochs

def test_minibatch_of_one_is_sgd_bitwise():
    cfg, p, params = _problem("cfg1")
    order = item_order(p.n_items, 77, 0)
    a, b = params.copy(), params.copy()
    oracle.sgd_epoch(a, p, order, 0.01)
    oracle.minibatch_epoch(b, p, order, 1, 0.01)
    for x, y in zip(a.U + [a.G] + a.V, b.U + [b.G] + b.V):
        assert np.array_equal(x, y)


def test_full_batch_is_a_gradient_step():
    cfg, p, params = _problem("tiny3")
    order = item_order(p.n_items, 5, 0)
    eta = 0.003
    dU, dG, dV = oracle.full_grad(params, p)
    b = params.copy()
    oracle.minibatch_epoch(b, p, order, p.n_items, eta)
    for x, x0, g in zip(b.U + [b.G] + b.V, params.U + [params.G] + params.V, dU + [dG] + dV):
        assert rel(x, x0 - eta * g) < 1e-13


def test_partial_minibatch_range_composes():
    cfg, p, params = _problem("cfg1")
    order = item_order(p.n_items, 9, 0)
    a, b = params.copy(), params.copy()
    oracle.minibatch_epoch(a, p, order, 500, 0.01)
    nb = oracle.minibatch_epoch(b, p, order, 500, 0.01, 0, 4)
    assert nb == 4
    oracle.minibatch_epoch(b, p, order, 500, 0.01, 4, -1)
    for x, y in zip(a.U + [a.G] + a.V, b.U + [b.G] + b.V):
        assert np.array_equal(x, y)


def test_single_item_step_descends_its_term():
    rng = np.random.default_rng(8)
    dims, ranks = (4, 3, 5), (2, 3, 2)
    params = _rand_params(rng, dims, ranks, [])
    rows = [1, 2, 3]
    reg_row, reg_core, x = np.array([0.1, 0.2, 0.3]), 0.01, 4.0
    before = item_phi(params.U, params.G, rows, x, reg_row, reg_core)
    e, gU, gG = oracle.tensor_item_grad(params, rows, x, reg_row, reg_core)
    for n in range(3):
        params.U[n][rows[n]] -= 1e-3 * gU[n]
    params.G -= 1e-3 * gG
    after = item_phi(params.U, params.G, rows, x, reg_row, reg_core)
    assert after < before


def test_full_batch_descent_is_monotone():
    cfg, p, params = _problem("cfg1")
    order = item_order(p.n_items, 1, 0)
    prev = oracle.loss(params, p)[0]
    for _ in range(5):
        oracle.minibatch_epoch(params, p, order, p.n_items, 0.002)
        cur = oracle.loss(params, p)[0]
        assert cur <= prev
        prev = cur


def test_sgd_learns_planted_signal():
    cfg = get_config("cfg1", planted=True, nnz=20000)
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    params = oracle.Params.from_arrays(U, G, V, [0])
    r0 = oracle.rmse(params, p.test_idx, p.test_val)
    assert abs(r0 - np.sqrt(np.mean(p.test_val ** 2))) < 0.05  # untrained ~ sqrt(mean x^2)
    # from the small N(0, 0.1) start SGD first sits near the saddle at zero
    # for about ten epochs, then drops to the noise level
    for ep in range(20):
        oracle.sgd_epoch(params, p, item_order(p.n_items, 3, ep), oracle.eta_at(0.01, 0.1, ep))
    r = oracle.rmse(params, p.test_idx, p.test_val)
    spread = np.std(p.test_val)
    assert r < 0.8 * spread, (r, spread)


def test_uncoupled_epoch_ignores_matrix_parameters():
    cfg = get_config("tiny3")
    cfg = cfg.scaled(matrices=())
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    params = oracle.Params.from_arrays(U, G, V, [])
    before = oracle.loss(params, p)[0]
    oracle.sgd_epoch(params, p, item_order(p.n_items, 0, 0), 0.01)
    assert oracle.loss(params, p)[0] < before


# ---------------------------------------------------------------- adjoint

def test_adjoint_matches_finite_differences():
    cfg, p, _ = _problem("tiny3")
    rng = np.random.default_rng(9)
    params = _rand_params(rng, cfg.dims, cfg.ranks, [(s.mode, s.cols) for s in cfg.matrices], 0.6)
    gx = rng.normal(size=p.n_train)
    gy = [rng.normal(size=len(v)) for v in p.mat_val]
    mats = [(p.mat_row[m], p.mat_col[m]) for m in range(len(p.mat_val))]
    dU, dG, dV = oracle.adjoint(params, p.train_idx, gx, mats, gy)

    def L():
        val = gx @ dense_predict(params.U, params.G, p.train_idx)
        for m, (r, c) in enumerate(mats):
            cm = params.modes[m]
            val += gy[m] @ np.sum(params.U[cm][r] * params.V[m][c], axis=1)
        return val

    for n in range(cfg.order):
        assert rel(dU[n], fd_grad(L, params.U[n])) < 1e-7
    assert rel(dG, fd_grad(L, params.G)) < 1e-7
    assert rel(dV[0], fd_grad(L, params.V[0])) < 1e-7


# ---------------------------------------------------------------- QR (Alg 1 end)

def test_qr_step_keeps_predictions_and_orthogonalises():
    cfg, p, params = _problem("tiny4")
    q = oracle.qr_orthogonalize(params)
    grid = np.stack(np.meshgrid(*[np.arange(I) for I in cfg.dims], indexing="ij")).reshape(cfg.order, -1)
    assert rel(dense_tucker(q.U, q.G), dense_tucker(params.U, params.G)) < 1e-12
    for u in q.U:
        assert np.allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)
    for m, c in enumerate(params.modes):
        assert rel(q.U[c] @ q.V[m].T, params.U[c] @ params.V[m].T) < 1e-12
    assert rel(oracle.predict(q, grid), oracle.predict(params, grid)) < 1e-12


# ---------------------------------------------------------------- damped batches

def test_leave_one_out_contraction_is_prediction_gradient():
    # w_n = G x_{-n} {u} is the derivative of the prediction w.r.t. row n (Eq 4)
    rng = np.random.default_rng(11)
    for dims, ranks in [((4, 3, 5), (2, 3, 2)), ((3, 2, 2, 3), (2, 2, 1, 2))]:
        params = _rand_params(rng, dims, ranks, [])
        rows = [int(rng.integers(0, I)) for I in dims]
        w = oracle.tensor_item_w(params, rows)
        for n in range(len(dims)):
            def pred():
                return dense_predict(params.U, params.G, np.array(rows)[:, None])[0]
            mask = np.zeros_like(params.U[n], dtype=bool)
            mask[rows[n]] = True
            assert rel(w[n], fd_grad(pred, params.U[n], mask=mask)[rows[n]]) < 1e-8


def test_damped_batches_reduce_to_sgd_for_small_steps():
    cfg, p, params = _problem("cfg1")
    order = item_order(p.n_items, 4, 0)
    a, b = params.copy(), params.copy()
    oracle.sgd_epoch(a, p, order, 0.01)
    oracle.minibatch_epoch(b, p, order, 1, 0.01, damping=True)
    for x, y in zip(a.U + [a.G] + a.V, b.U + [b.G] + b.V):
        assert np.array_equal(x, y)


def test_damped_step_of_one_entry():
    cfg, p, params = _problem("tiny3", matrices=(), nnz=12, dims=(10, 8, 9))
    cnt, _ = oracle.counts(params, p)
    e0 = 0
    rows = [int(p.train_idx[n][e0]) for n in range(3)]
    reg_row = [cfg.lambda_reg / cnt[n][rows[n]] for n in range(3)]
    reg_core = cfg.lambda_reg / p.n_train
    eta = 50.0  # large enough that every block is damped
    e, gU, gG = oracle.tensor_item_grad(params, rows, p.train_val[e0], reg_row, reg_core)
    w = oracle.tensor_item_w(params, rows)
    b = params.copy()
    order = np.arange(p.n_items)
    oracle.minibatch_epoch(b, p, order, 1, eta, 0, 1, damping=True)
    kappa = 4.0
    for n in range(3):
        L = w[n] @ w[n] + reg_row[n]
        step = eta / max(1.0, kappa * eta * L)
        assert rel(b.U[n][rows[n]], params.U[n][rows[n]] - step * gU[n]) < 1e-13
    LG = np.prod([params.U[n][rows[n]] @ params.U[n][rows[n]] for n in range(3)]) + reg_core
    assert rel(b.G, params.G - eta / max(1.0, kappa * eta * LG) * gG) < 1e-13


# ------------------------------------------------- CP (hyper-diagonal core)
# The CP special case (Section 3's S^3CMTF-CP) stores only the J diagonal
# values of the core.  Pins: the dense Kronecker model with the embedded
# diagonal core, finite differences, and the Tucker oracle's own gradients
# restricted to the diagonal.

def _embed(g, N):
    G = np.zeros((g.size,) * N)
    for r in range(g.size):
        G[(r,) * N] = g[r]
    return G


def _cp_params(rng, dims, J, mats, scale=0.7):
    U = [rng.normal(0, scale, size=(I, J)) for I in dims]
    g = rng.normal(0, scale, size=J)
    V = [rng.normal(0, scale, size=(K, J)) for (_, K) in mats]
    return oracle.Params.from_arrays(U, g, V, [c for c, _ in mats], cp=True)


@pytest.mark.parametrize("dims,J", [((4, 3, 5), 2), ((3, 2, 2, 3), 2), ((5, 4, 3), 3)])
def test_cp_predict_matches_dense_kronecker(dims, J):
    rng = np.random.default_rng(40)
    params = _cp_params(rng, dims, J, [])
    grid = np.stack(np.meshgrid(*[np.arange(I) for I in dims], indexing="ij")).reshape(len(dims), -1)
    got = oracle.predict(params, grid)
    want = dense_predict(params.U, _embed(params.G, len(dims)), grid)
    assert rel(got, want) < 1e-13


@pytest.mark.parametrize("dims,J", [((4, 3, 5), 2), ((3, 2, 2, 3), 3)])
def test_cp_item_grad_matches_fd(dims, J):
    rng = np.random.default_rng(41)
    params = _cp_params(rng, dims, J, [])
    N = len(dims)
    rows = [int(rng.integers(0, I)) for I in dims]
    x, reg_row, reg_core = 2.5, [0.03 * (n + 1) for n in range(N)], 0.07
    e, gU, gg = oracle.tensor_item_grad(params, rows, x, reg_row, reg_core)

    def phi():
        return item_phi(params.U, _embed(params.G, N), rows, x, reg_row, reg_core)

    for n in range(N):
        mask = np.zeros_like(params.U[n], dtype=bool)
        mask[rows[n]] = True
        fd = fd_grad(phi, params.U[n], mask=mask)[rows[n]]
        assert rel(gU[n], fd) < 1e-7
    assert rel(gg, fd_grad(phi, params.G)) < 1e-7
    assert abs(e - (x - dense_predict(params.U, _embed(params.G, N), np.array(rows)[:, None])[0])) < 1e-12


def test_cp_grads_are_the_tucker_grads_on_the_diagonal():
    rng = np.random.default_rng(42)
    cp = _cp_params(rng, (6, 5, 4), 3, [])
    tk = oracle.Params.from_arrays(cp.U, _embed(cp.G, 3), cp.V, cp.modes)
    rows, x, reg_row, reg_core = [2, 4, 1], 3.0, [0.1, 0.2, 0.3], 0.05
    e1, gU1, gg = oracle.tensor_item_grad(cp, rows, x, reg_row, reg_core)
    e2, gU2, gG = oracle.tensor_item_grad(tk, rows, x, reg_row, reg_core)
    assert abs(e1 - e2) < 1e-14
    for a, b in zip(gU1, gU2):
        assert rel(a, b) < 1e-14
    assert rel(gg, [gG[r, r, r] for r in range(3)]) < 1e-14


def _cp_problem(name, **kw):
    cfg = get_config(name, **kw)
    p = make_problem(cfg)
    U, G, V = init_params(cfg)
    g = np.array([G[(r,) * cfg.order] for r in range(cfg.ranks[0])])
    return cfg, p, oracle.Params.from_arrays(U, g, V, [s.mode for s in cfg.matrices], cp=True)


def test_cp_batch_of_one_is_sgd():
    cfg, p, params = _cp_problem("cfg1")
    order = item_order(p.n_items, 5, 0)
    a, b = params.copy(), params.copy()
    oracle.sgd_epoch(a, p, order, 0.01)
    oracle.minibatch_epoch(b, p, order, 1, 0.01, damping=True)
    for x, y in zip(a.U + [a.G] + a.V, b.U + [b.G] + b.V):
        assert np.array_equal(x, y)
    assert rel(a.G, params.G) > 0  # the core moved


def test_cp_damped_step_of_one_entry():
    cfg, p, params = _cp_problem("tiny3", matrices=(), nnz=12, dims=(10, 8, 9), ranks=(2, 2, 2))
    cnt, _ = oracle.counts(params, p)
    rows = [int(p.train_idx[n][0]) for n in range(3)]
    reg_row = [cfg.lambda_reg / cnt[n][rows[n]] for n in range(3)]
    reg_core = cfg.lambda_reg / p.n_train
    eta = 50.0
    e, gU, gg = oracle.tensor_item_grad(params, rows, p.train_val[0], reg_row, reg_core)
    b = params.copy()
    oracle.minibatch_epoch(b, p, np.arange(p.n_items), 1, eta, 0, 1, damping=True)
    u = [params.U[n][rows[n]] for n in range(3)]
    # curvature of x~ in the diagonal core values: sum_r prod_n u_n[r]^2
    LG = sum(np.prod([u[n][r] ** 2 for n in range(3)]) for r in range(2)) + reg_core
    assert rel(b.G, params.G - eta / max(1.0, 4.0 * eta * LG) * gg) < 1e-13
    for n in range(3):
        w = params.G * np.prod([u[m] for m in range(3) if m != n], axis=0)
        step = eta / max(1.0, 4.0 * eta * (w @ w + reg_row[n]))
        assert rel(b.U[n][rows[n]], u[n] - step * gU[n]) < 1e-13


def test_cp_qr_is_rejected():
    rng = np.random.default_rng(43)
    with pytest.raises(ValueError):
        oracle.qr_orthogonalize(_cp_params(rng, (5, 4, 3), 2, []))


# ------------------------------------- batched epochs against a restatement
# The damped mini-batch rule (several entries per row, matrix rows on both
# sides, the per-batch reset of sums and curvatures, the hyper-diagonal
# core) against tests/dense_ref.damped_batch_step, which restates Eq (8) and
# the damping reading with np.einsum and per-block dictionaries.

def _cp_of(params, J):
    U = [u[:, :J].copy() for u in params.U]
    V = [v[:, :J].copy() for v in params.V]
    g = np.linspace(0.4, -0.3, J)
    return oracle.Params.from_arrays(U, g, V, params.modes, cp=True)


@pytest.mark.parametrize("name,eta,batch,cp,damping", [
    ("tiny3", 5.0, 13, False, True),
    ("tiny4", 5.0, 9, False, True),
    ("cfg1", 2.0, 700, False, True),
    ("tiny3", 5.0, 13, True, True),
    ("tiny4", 5.0, 9, True, True),
    ("tiny3", 0.02, 13, False, False),
    ("cfg1", 0.002, 700, False, False),
])
def test_batched_epoch_matches_independent_restatement(name, eta, batch, cp, damping):
    cfg, p, params = _problem(name)
    if cp:
        params = _cp_of(params, min(cfg.ranks))
    cnt, cntV = oracle.counts(params, p)
    order = item_order(p.n_items, 5, 0)
    got = params.copy()
    oracle.minibatch_epoch(got, p, order, batch, eta, 0, 3, damping=damping)
    U, G, V = params.U, params.G, params.V
    mats = [(p.mat_row[m], p.mat_col[m], p.mat_val[m]) for m in range(len(p.mat_val))]
    damped = 0
    for b in range(3):
        items = order[b * batch:(b + 1) * batch]
        U, G, V, nd = damped_batch_step(U, G, V, params.modes, items, (p.train_idx, p.train_val), mats, eta,
                                        cfg.lambda_reg, cfg.lambda_m, cnt, cntV, p.n_train, damping=damping,
                                        cp=cp)
        damped += nd
    if damping:
        assert damped > 0  # the rule is exercised, not just plain SGD sums
    for a, b_ in zip(got.U + [got.G] + got.V, U + [G] + V):
        assert rel(a, b_) < 1e-13
        assert np.max(np.abs(a - b_)) <= 1e-13 * max(1.0, np.max(np.abs(b_)))


def test_threaded_batched_epoch_is_bitwise_sequential():
    for name, cp in [("tiny3", False), ("tiny4", False), ("cfg1", False), ("cfg5_slice", False), ("tiny4", True)]:
        cfg, p, params = _problem(name)
        if cp:
            params = _cp_of(params, 1)
        order = item_order(p.n_items, 3, 0)[:3000]
        for damping, eta in [(True, 0.5), (False, 0.01)]:
            for batch in (1, 7, 500, 10 ** 9):
                # the worker threads start once per batch: 300 items are
                # already 300 or 43 batches at the two smallest sizes
                o = order[:300] if batch < 500 else order
                ref = params.copy()
                oracle.minibatch_epoch(ref, p, o, batch, eta, damping=damping)
                for threads in (2, 5):
                    got = params.copy()
                    oracle.minibatch_epoch(got, p, o, batch, eta, damping=damping, threads=threads)
                    for a, b in zip(got.U + [got.G] + got.V, ref.U + [ref.G] + ref.V):
                        assert np.array_equal(a, b)


def test_matrix_predict_is_row_dot_products():
    rng = np.random.default_rng(21)
    for J in (1, 3, 10, 16):
        params = _rand_params(rng, (30, 4, 5), (J, 2, 2), [(0, 25)])
        row = rng.integers(0, 30, size=200)
        col = rng.integers(0, 25, size=200)
        want = np.einsum("ij,ij->i", params.U[0][row], params.V[0][col])
        got = oracle.matrix_predict(params, 0, row, col)
        assert rel(got, want) < 1e-15
