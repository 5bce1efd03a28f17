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
