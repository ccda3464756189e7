"""Chebyshev moments of the DOS and LDOS (Sec. 3.1).

Definitions followed:
* DOS (Sec. 2.2, eqn dos): mu = (1/N) sum_i delta(lambda - lambda_i).
* Chebyshev three-term recurrence (eq. cheb_3term):
  T_0 = 1, T_1 = x, T_{m+1} = 2 x T_m - T_{m-1}.
* DOS moments (eqn doscoeff): d_m = (1/N) tr T_m(H) = (1/N) sum_i T_m(lambda_i).
  (The printed right-hand side omits the 1/N on the trace; the middle
  expression fixes it.)
* PDOS moments (eqn pdoscoeff): d_mk = T_m(H)_kk = sum_i q_i(k)^2 T_m(lambda_i).
* Hutchinson / Bekas estimators (eq. probe_trace, eq. probe_diag):
  E[z^T B z] = tr B and E[z o Bz] = diag B for i.i.d. zero-mean unit-variance z;
  with N_z probes the moments cost one sparse product per term and probe.

Index convention: "M moments" means T_0 .. T_{M-1}, i.e. M-1 applications of H.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def cheb_of_eigs(lam: np.ndarray, M: int) -> np.ndarray:
    """[M][len(lam)] table T_m(lambda_i) = cos(m arccos lambda_i)."""
    th = np.arccos(np.clip(lam, -1.0, 1.0))
    return np.cos(np.outer(np.arange(M), th))


def exact_moments_eig(H, M: int):
    """Exact DOS moments d_m and PDOS moments d_mk from a dense symmetric
    eigendecomposition H = Q Lambda Q^T (eqn doscoeff, eqn pdoscoeff).
    Returns (mu [M], ldos [N][M])."""
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H, dtype=np.float64)
    lam, Q = np.linalg.eigh(Hd)
    T = cheb_of_eigs(lam, M)                 # [M][N]
    mu = T.mean(axis=1)
    ldos = (Q * Q) @ T.T                     # sum_i Q_ki^2 T_m(lambda_i)
    return mu, ldos


def exact_moments_recurrence(H, M: int):
    """Exact moments by running the recurrence on Z = I (every basis vector as
    a probe): T_m(H) itself, column block by column block.  Returns
    (mu [M], ldos [N][M])."""
    H = sp.csr_matrix(H)
    N = H.shape[0]
    ldos = np.zeros((N, M))
    B = 512
    for c0 in range(0, N, B):
        c1 = min(N, c0 + B)
        Z = np.zeros((N, c1 - c0))
        Z[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        for m, Y in enumerate(cheb_vectors(H, Z, M)):
            ldos[c0:c1, m] = Y[np.arange(c0, c1), np.arange(c1 - c0)]
    return ldos.mean(axis=0), ldos


def cheb_vectors(H, Z: np.ndarray, M: int):
    """Yield Y_m = T_m(H) Z for m = 0..M-1 by the three-term recurrence."""
    if M <= 0:
        return
    Yprev = np.array(Z, dtype=np.float64, copy=True)
    yield Yprev
    if M == 1:
        return
    Y = H @ Yprev
    yield Y
    for _ in range(2, M):
        Ynext = 2.0 * (H @ Y) - Yprev
        Yprev, Y = Y, Ynext
        yield Y


def stochastic_moments(H, Z: np.ndarray, M: int, ldos: bool = True):
    """Probe estimates with the given probe block Z [N][k] (fp64 values):

        mu_pp[j][m] = (1/N) z_j^T T_m(H) z_j          (per probe)
        mu[m]       = mean_j mu_pp[j][m]              (eq. probe_trace, / N)
        C[i][m]     = (1/k) sum_j z_ij (T_m(H) z_j)_i  (eq. probe_diag)

    Returns (mu [M], mu_pp [k][M], C [N][M] or None)."""
    N, k = Z.shape
    mu_pp = np.zeros((k, M))
    C = np.zeros((N, M)) if ldos else None
    for m, Y in enumerate(cheb_vectors(H, Z, M)):
        P = Z * Y
        mu_pp[:, m] = P.sum(axis=0) / N
        if ldos:
            C[:, m] = P.mean(axis=1)
    return mu_pp.mean(axis=0), mu_pp, C


def cheb_at_zero(M: int) -> np.ndarray:
    """T_m(0) = cos(m pi / 2): 1, 0, -1, 0, ..."""
    return np.array([(1.0, 0.0, -1.0, 0.0)[m % 4] for m in range(M)])


def power_moment_2(g) -> float:
    """tr(H^2)/N = (1/N) sum_ij A_ij^2 / (d_i d_j): the second *power* moment."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    d = g.deg.astype(np.float64)
    return float(np.sum(1.0 / (d[rows] * d[g.col])) / g.n)


def cheb_moment_2_diag(g) -> np.ndarray:
    """diag T_2(H)_ii = 2 sum_j A_ij / (d_i d_j) - 1 (closed form, T_2 = 2x^2 - 1)."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    d = g.deg.astype(np.float64)
    s = np.bincount(rows, weights=1.0 / (d[rows] * d[g.col]), minlength=g.n)
    return 2.0 * s - 1.0


def cv_ldos(H, Z: np.ndarray, M: int, G: np.ndarray):
    """Diagonal control variate diag(g_m) per moment (learned part; not in the
    paper).  Per probe and node the estimate is
        g_im + z_ij ((T_m(H) - diag g_m) z_j)_i = g_im (1 - z_ij^2) + z_ij (T_m z_j)_i,
    which stays unbiased for any fixed g.  Averaged over the k probes.
    Returns (mu [M] = mean over nodes, C [N][M], S2 [N][M]) where S2 is the
    mean over probes of the squared per-probe estimate (for variances)."""
    N, k = Z.shape
    C = np.zeros((N, M))
    S2 = np.zeros((N, M))
    zz = Z * Z
    for m, Y in enumerate(cheb_vectors(H, Z, M)):
        est = G[:, m:m + 1] * (1.0 - zz) + Z * Y
        C[:, m] = est.mean(axis=1)
        S2[:, m] = (est * est).mean(axis=1)
    return C.mean(axis=0), C, S2


def ldos_probe_variance(exact_ldos: np.ndarray, M: int, kind: str, g: np.ndarray | None = None):
    """Per-probe variance of the node-i, moment-m diagonal estimate for a
    single probe, from exact PDOS moments b = d_mi and d_{2m,i}
    (uses T_m^2 = (T_{2m} + I)/2, so needs exact_ldos up to 2M-2):

        Rademacher (with or without a diagonal CV): (1 + d_{2m,i})/2 - b^2
        Gaussian, plain:                            (1 + d_{2m,i})/2 - b^2 + 2 b^2
        Gaussian with diagonal CV g:                (1 + d_{2m,i})/2 - b^2 + 2 (b - g)^2

    Derivation: for symmetric B, z_i (Bz)_i = B_ii z_i^2 + z_i sum_{j!=i} B_ij z_j;
    the cross term has variance sum_{j!=i} B_ij^2 = (B^2)_ii - b^2 and is
    uncorrelated with the first; Var(z_i^2) is 0 (Rademacher) or 2 (Gaussian),
    and the control variate replaces b by b - g in the first term.
    Returns [N][M]."""
    b = exact_ldos[:, :M]
    d2 = exact_ldos[:, [2 * m for m in range(M)]]
    vr = 0.5 * (1.0 + d2) - b * b
    if kind == "rademacher":
        return vr
    if kind == "gaussian":
        if g is None:
            return vr + 2.0 * b * b
        return vr + 2.0 * (b - g[:, :M]) ** 2
    raise ValueError(kind)
