"""Learned control variate (not in the paper; parity unpinned by the paper).

A small per-node MLP predicts g_i = (g_i0 .. g_i,M-1), an estimate of the PDOS
moments T_m(H)_ii, from cheap structural features; the diagonal estimator
becomes  g_im + z_i ((T_m(H) - diag g_m) z)_i  (see :func:`oracle.kpm.cv_ldos`),
unbiased for any g.  This module is the fp64 reference for:

* node features (5 per node), log1p-scaled:
    degree d_i; mean and max neighbour degree; local clustering
    2 t_i / (d_i (d_i - 1)) (0 when d_i < 2, t_i = triangles through i);
    number of distinct nodes at distance exactly 2;
* the MLP 5 -> 128 -> 128 -> 64 (ReLU, ReLU, linear), flat fp32 parameter
  vector laid out [W1 (5x128, row-major in x out), b1, W2, b2, W3, b3];
* mean-squared-error loss, its gradient, and the Adam update
  (Kingma & Ba, ICLR 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
"""
from __future__ import annotations

import numpy as np

N_FEAT = 5
WIDTH = 128
N_OUT = 64
SHAPES = [(N_FEAT, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, N_OUT), (N_OUT,)]


def n_params(n_out: int = N_OUT) -> int:
    return N_FEAT * WIDTH + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH * n_out + n_out


def unpack(params: np.ndarray, n_out: int = N_OUT):
    shapes = [(N_FEAT, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, n_out), (n_out,)]
    out, o = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(np.asarray(params[o:o + size], dtype=np.float64).reshape(s))
        o += size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def raw_features(g) -> np.ndarray:
    """[N][5] raw (unscaled) features from the CSR graph (scipy products)."""
    import scipy.sparse as sp
    n = g.n
    d = g.deg.astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    A = sp.csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr), shape=(n, n))
    nd = d[g.col]
    nmean = np.bincount(rows, weights=nd, minlength=n) / d
    nmax = np.zeros(n)
    np.maximum.at(nmax, rows, nd)
    A2 = (A @ A).tocsr()
    tri = np.asarray(A.multiply(A2).sum(axis=1)).ravel() / 2.0
    clus = np.where(d >= 2, 2.0 * tri / np.maximum(d * (d - 1), 1.0), 0.0)
    # distinct nodes at distance exactly 2: pattern of A^2, minus self, minus N(i)
    P2 = A2.copy()
    P2.data[:] = 1.0
    P2 = P2 - P2.multiply(A) - sp.diags(P2.diagonal())
    P2.eliminate_zeros()
    two_hop = np.diff(P2.tocsr().indptr).astype(np.float64)
    return np.stack([d, nmean, nmax, clus, two_hop], axis=1)


def raw_features_bruteforce(g) -> np.ndarray:
    """Same features with Python sets, for tiny graphs."""
    nb = [set(g.neighbors(i).tolist()) for i in range(g.n)]
    out = np.zeros((g.n, N_FEAT))
    for i in range(g.n):
        d = len(nb[i])
        nd = [len(nb[j]) for j in nb[i]]
        tri = sum(1 for a in nb[i] for b in nb[i] if a < b and b in nb[a])
        two = set()
        for j in nb[i]:
            two |= nb[j]
        two -= nb[i]
        two.discard(i)
        out[i] = [d, np.mean(nd), max(nd), (2.0 * tri / (d * (d - 1)) if d >= 2 else 0.0), len(two)]
    return out


def log_scale(raw: np.ndarray) -> np.ndarray:
    return np.log1p(raw)


def standardize(x: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    return (x - mean[None, :]) / std[None, :]


def forward(params: np.ndarray, x: np.ndarray, n_out: int = N_OUT, keep: bool = False):
    W1, b1, W2, b2, W3, b3 = unpack(params, n_out)
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    out = h2 @ W3 + b3
    if keep:
        return out, (x, a1, h1, a2, h2)
    return out


def mse(params, x, target, n_out: int = N_OUT) -> float:
    out = forward(params, x, n_out)
    return float(np.mean((out - target) ** 2))


def mse_grad(params, x, target, n_out: int = N_OUT):
    """(loss, flat gradient) of mean((f(x) - target)^2) over nodes and outputs."""
    W1, b1, W2, b2, W3, b3 = unpack(params, n_out)
    out, (x, a1, h1, a2, h2) = forward(params, x, n_out, keep=True)
    r = out - target
    loss = float(np.mean(r * r))
    d3 = 2.0 * r / r.size
    gW3 = h2.T @ d3
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3.T) * (a2 > 0)
    gW2 = h1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (a1 > 0)
    gW1 = x.T @ d1
    gb1 = d1.sum(axis=0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(params, m, v, grad, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step count t >= 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
