"""Independent dense references used to pin the oracle (tests only).

Nothing here calls the oracle or the library: the Tucker model is rebuilt
densely from the Kronecker identity vec(G x_1 U1 ... x_N UN) =
(UN kron ... kron U1) vec(G) with column-major vec (Kolda and Bader), and
gradients are taken by central finite differences of the per-item terms.
"""
import numpy as np


def dense_tucker(U, G):
    """Full reconstruction X~ (I_1 x ... x I_N) via the Kronecker identity."""
    kr = U[-1]
    for u in reversed(U[:-1]):
        kr = np.kron(kr, u)
    x = kr @ np.asarray(G).flatten(order="F")
    return x.reshape([u.shape[0] for u in U], order="F")


def dense_predict(U, G, idx):
    return dense_tucker(U, G)[tuple(np.asarray(idx))]


def item_phi(U, G, rows, x, reg_row, reg_core):
    """Half of one tensor entry's share of f_t (Eq 7): the quantity whose
    gradient the per-entry formulas give."""
    X = dense_tucker(U, G)
    e = x - X[tuple(rows)]
    val = 0.5 * e * e + 0.5 * reg_core * float(np.sum(np.asarray(G) ** 2))
    for n, r in enumerate(rows):
        val += 0.5 * reg_row[n] * float(np.sum(U[n][r] ** 2))
    return val


def fd_grad(fun, arr, h=1e-6, mask=None):
    """Central differences of scalar fun() w.r.t. every entry of arr (in place)."""
    g = np.zeros_like(arr)
    flat = arr.reshape(-1)
    gf = g.reshape(-1)
    sel = range(flat.size) if mask is None else np.flatnonzero(np.asarray(mask).reshape(-1))
    for k in sel:
        old = flat[k]
        step = h * max(1.0, abs(old))
        flat[k] = old + step
        fp = fun()
        flat[k] = old - step
        fm = fun()
        flat[k] = old
        gf[k] = (fp - fm) / (2 * step)
    return g


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    d = np.linalg.norm(a - b)
    s = max(np.linalg.norm(b), 1e-300)
    return d / s


# ------------------------------------------------------------------------
# An independent restatement of the damped mini-batch step (Eq 8 for the
# per-entry gradients; the curvature damping reading for the step), used to
# pin the oracle's batched epoch.  It shares nothing with the oracle's code:
# predictions and leave-one-out contractions are np.einsum calls on the whole
# core, gradients are summed per parameter block in Python dictionaries.

_LETTERS = "abcdefgh"


def _contract(G, rows, skip=None):
    """G x_1 rows[0] ... x_N rows[N-1], leaving mode `skip` uncontracted."""
    N = G.ndim
    spec = _LETTERS[:N] + "," + ",".join(_LETTERS[n] for n in range(N) if n != skip)
    spec += "->" + ("" if skip is None else _LETTERS[skip])
    return np.einsum(spec, G, *[rows[n] for n in range(N) if n != skip])


def _outer(rows):
    out = rows[0]
    for r in rows[1:]:
        out = np.multiply.outer(out, r)
    return out


def damped_batch_step(U, G, V, modes, items, tensor, mats, eta, lambda_reg, lambda_m,
                      cnt, cntV, n_train, damping=True, cp=False):
    """One batch: every item's gradient at the batch-start values, summed per
    block (factor row, coupled-factor row, core) with its curvature L, then
    block <- block - eta / max(1, (N + 1) eta L) * sum (damping) or
    - eta * sum.  tensor = (idx [N][nnz], val); mats[m] = (row, col, val);
    items are ids (tensor entries first, then each matrix's entries).
    cp: G holds the J diagonal values of a hyper-diagonal core.  Returns new
    (U, G, V, number of blocks whose step the damping shortened)."""
    N = len(U)
    Gd = G
    if cp:
        J = G.shape[0]
        Gd = np.zeros((J,) * N)
        for r in range(J):
            Gd[(r,) * N] = G[r]
    idx, val = tensor
    nX = val.shape[0]
    starts = [nX]
    for (r, _, _) in mats:
        starts.append(starts[-1] + len(r))
    gsum, Lsum = {}, {}

    def add(key, g, L):
        if key in gsum:
            gsum[key] = gsum[key] + g
            Lsum[key] = Lsum[key] + L
        else:
            gsum[key] = g.copy()
            Lsum[key] = L

    reg_core = lambda_reg / n_train
    for t in items:
        t = int(t)
        if t < nX:
            rows_i = [int(idx[n][t]) for n in range(N)]
            rows = [U[n][rows_i[n]] for n in range(N)]
            e = val[t] - float(_contract(Gd, rows))
            for n in range(N):
                w = _contract(Gd, rows, skip=n)
                reg = lambda_reg / cnt[n][rows_i[n]]
                add(("U", n, rows_i[n]), -e * w + reg * rows[n], float(w @ w) + reg)
            op = _outer(rows)
            if cp:
                d = np.array([op[(r,) * N] for r in range(G.shape[0])])
                add(("G",), -e * d + reg_core * G, float(d @ d) + reg_core)
            else:
                add(("G",), -e * op + reg_core * G, float(np.prod([r @ r for r in rows])) + reg_core)
        else:
            m = max(k for k in range(len(mats)) if t >= starts[k])
            e_i = t - starts[m]
            r, c, y = mats[m]
            ri, ci = int(r[e_i]), int(c[e_i])
            u, v = U[modes[m]][ri], V[m][ci]
            e = y[e_i] - float(u @ v)
            rv = lambda_m * lambda_reg / cntV[m][ci]
            add(("U", modes[m], ri), -lambda_m * e * v, lambda_m * float(v @ v))
            add(("V", m, ci), -lambda_m * e * u + rv * v, lambda_m * float(u @ u) + rv)
    U2, G2, V2 = [u.copy() for u in U], G.copy(), [v.copy() for v in V]
    kappa = N + 1
    n_damped = 0
    for key, g in gsum.items():
        step = eta / max(1.0, kappa * eta * Lsum[key]) if damping else eta
        n_damped += int(step < eta)
        if key[0] == "U":
            U2[key[1]][key[2]] -= step * g
        elif key[0] == "V":
            V2[key[1]][key[2]] -= step * g
        else:
            G2 = G2 - step * g
    return U2, G2, V2, n_damped
