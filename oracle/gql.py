"""Gauss quadrature and Lanczos, GQL (Sec. 3.2).

Oracle: test infrastructure only (tests, the smoke check and the CPU baseline
of the benchmark use it; the GPU library never does).

For a probe z, K Lanczos steps on H from v_1 = z / |z| give the tridiagonal
matrix Gamma_K (diagonal alpha_1..alpha_K, off-diagonal beta_1..beta_{K-1})
with H V_K = V_K Gamma_K + r e_K^T.  With (tau_i, p_i) the eigenpairs of
Gamma_K, z^T f(H) z is approximated by |z|^2 sum_i p_{1i}^2 f(tau_i) -- the
K-node Gauss rule of the measure sum_i (q_i^T z)^2 delta(lambda - lambda_i),
exact for polynomials of degree <= 2K - 1.  Averaged over probes and divided
by N, the point masses estimate the DOS; converted to Chebyshev moments they
equal the KPM estimates of the same probes for m <= 2K - 1.

Lanczos here is the plain three-term recurrence in fp64 (no
reorthogonalization), stopping early when beta falls below `tol` (an
invariant subspace has been found: the Gauss rule is then exact).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos(H, z: np.ndarray, K: int, tol: float = 1e-10):
    """(alpha [K'], beta [K'-1]) for K' <= K steps from v_1 = z / |z|."""
    v = np.asarray(z, dtype=np.float64) / np.linalg.norm(z)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alpha, beta = [], []
    for k in range(K):
        w = H @ v - b_prev * v_prev
        a = float(v @ w)
        w = w - a * v
        alpha.append(a)
        b = float(np.linalg.norm(w))
        if k == K - 1 or b < tol:
            break
        beta.append(b)
        v_prev, v, b_prev = v, w / b, b
    return np.array(alpha), np.array(beta)


def quadrature(alpha: np.ndarray, beta: np.ndarray):
    """Nodes tau_i (ascending) and weights p_{1i}^2 of the Gauss rule of
    Gamma (Golub-Welsch: eigenvalues and first eigenvector components)."""
    if alpha.size == 1:
        return alpha.copy(), np.ones(1)
    tau, P = eigh_tridiagonal(alpha, beta)
    return tau, P[0, :] ** 2


def gql_probes(H, Z: np.ndarray, K: int):
    """Per probe j: nodes [K'_j] and weights [K'_j] scaled by |z_j|^2 / N."""
    n = Z.shape[0]
    out = []
    for j in range(Z.shape[1]):
        a, b = lanczos(H, Z[:, j], K)
        tau, w = quadrature(a, b)
        out.append((tau, w * float(Z[:, j] @ Z[:, j]) / n))
    return out


def gql_moments(rules, M: int) -> np.ndarray:
    """mu_m = (1/k) sum_j sum_i w_ji T_m(tau_ji), m = 0..M-1."""
    mu = np.zeros(M)
    m = np.arange(M)
    for tau, w in rules:
        T = np.cos(np.outer(m, np.arccos(np.clip(tau, -1.0, 1.0))))
        mu += T @ w
    return mu / len(rules)


def gql_histogram(rules, n_bins: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """The averaged point masses binned like the other histograms (half-open
    bins, last closed).  Nodes are clamped to [-1, 1], the interval holding
    the spectrum of H: a rule computed in finite precision can place the node
    of the eigenvalue 1 (or -1) a rounding error outside it."""
    from .reconstruct import bin_edges, spike_bin
    e = bin_edges(n_bins, lo, hi)
    h = np.zeros(n_bins)
    for tau, w in rules:
        for t, x in zip(tau, w):
            b = spike_bin(min(max(float(t), -1.0), 1.0), e)
            if b is not None:
                h[b] += x
    return h / len(rules)
