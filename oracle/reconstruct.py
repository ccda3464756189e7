"""Density reconstruction from Chebyshev moments (Sec. 2.2, 3.1, 4.1).

* Orthogonality (eqn orth): T_m and T_n are orthogonal on [-1, 1] under the
  weight 1/(pi sqrt(1-x^2)), with norm 1 for m = n = 0 and 1/2 otherwise
  (the printed weight carries a Kronecker delta in n; this is its reading).
* Series (eqn doscoeff, read with the sum from m = 0):
      rho(x) = [g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)] / (pi sqrt(1 - x^2)).
* Jackson damping (Sec. 4.1, Jackson's theorem): the truncated series is
  multiplied by the Jackson factors.  The paper names them without giving
  them; the standard kernel for M moments (Weisse, Wellein, Alvermann &
  Fehske, Rev. Mod. Phys. 78, 2006, the KPM review the paper cites) is
      g_m = [(M - m + 1) cos(pi m/(M+1)) + sin(pi m/(M+1)) cot(pi/(M+1))] / (M+1).
* Spectral histogram (Sec. 2.2, after eqn reg_dos): the density integrated
  over equal bins.  With theta = arccos x, the mass of [a, b] is
      (1/pi) [g_0 mu_0 (theta_a - theta_b)
              + 2 sum_{m>=1} g_m mu_m (sin m theta_a - sin m theta_b) / m].
  Bins are half-open [e_b, e_{b+1}), the last one closed; e_b = lo + (hi-lo) b / n_bins.
  Point masses (filtered spikes) are added to the bin that contains them.
* Density points: the K Chebyshev nodes x_k = cos(pi (k + 1/2) / K).
"""
from __future__ import annotations

import numpy as np


def jackson(M: int) -> np.ndarray:
    m = np.arange(M, dtype=np.float64)
    a = np.pi / (M + 1)
    return ((M - m + 1) * np.cos(a * m) + np.sin(a * m) / np.tan(a)) / (M + 1)


def damping(M: int, kernel: str) -> np.ndarray:
    if kernel == "jackson":
        return jackson(M)
    if kernel == "none":
        return np.ones(M)
    raise ValueError(kernel)


def bin_edges(n_bins: int, lo: float, hi: float) -> np.ndarray:
    return np.array([lo + (hi - lo) * b / n_bins for b in range(n_bins + 1)])


def histogram(mu: np.ndarray, n_bins: int, lo: float = -1.0, hi: float = 1.0,
              kernel: str = "jackson", spikes=()) -> np.ndarray:
    """Bin masses of the reconstructed density for each row of mu [rows][M]
    (or a single [M] vector), plus point masses `spikes` = [(lambda, weight)]."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    M = mu.shape[1]
    c = mu * damping(M, kernel)[None, :]
    e = bin_edges(n_bins, lo, hi)
    th = np.arccos(np.clip(e, -1.0, 1.0))
    m = np.arange(1, M)
    # F(theta) = g_0 mu_0 theta + 2 sum_{m>=1} g_m mu_m sin(m theta)/m; mass = (F(th_a) - F(th_b))/pi
    S = np.sin(np.outer(th, m)) / m[None, :]                  # [edges][M-1]
    F = np.outer(c[:, 0], th) + 2.0 * c[:, 1:] @ S.T           # [rows][edges]
    hist = (F[:, :-1] - F[:, 1:]) / np.pi
    for lam, w in spikes:
        b = spike_bin(lam, e)
        if b is not None:
            hist[:, b] += w
    return hist


def spike_bin(lam: float, edges: np.ndarray):
    n_bins = len(edges) - 1
    if lam < edges[0] or lam > edges[-1]:
        return None
    b = int(np.searchsorted(edges, lam, side="right")) - 1
    return min(max(b, 0), n_bins - 1)


def cheb_nodes(K: int) -> np.ndarray:
    return np.cos(np.pi * (np.arange(K) + 0.5) / K)


def density(mu: np.ndarray, x: np.ndarray, kernel: str = "jackson") -> np.ndarray:
    """rho(x) for each row of mu, by direct summation of the damped series."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    M = mu.shape[1]
    c = mu * damping(M, kernel)[None, :]
    x = np.asarray(x, dtype=np.float64)
    T = np.cos(np.outer(np.arange(M), np.arccos(np.clip(x, -1.0, 1.0))))  # [M][K]
    w = np.full(M, 2.0)
    w[0] = 1.0
    return (c * w[None, :]) @ T / (np.pi * np.sqrt(1.0 - x * x))[None, :]


def exact_histogram(eigs: np.ndarray, n_bins: int, lo: float = -1.0, hi: float = 1.0,
                    snap: float = 1e-9) -> np.ndarray:
    """Histogram of exact eigenvalues (mass 1/N each), with values within
    `snap` of an edge moved onto it before binning."""
    e = bin_edges(n_bins, lo, hi)
    lam = np.array(eigs, dtype=np.float64, copy=True)
    for b in range(len(e)):
        lam[np.abs(lam - e[b]) <= snap] = e[b]
    h = np.zeros(n_bins)
    for v in lam:
        b = spike_bin(v, e)
        if b is not None:
            h[b] += 1.0 / len(lam)
    return h
