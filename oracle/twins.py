"""Twin motifs and probe projection (Sec. 3.4, motif filtering).

Two nodes with identical open neighbourhoods ("node copies", e.g. two dangling
nodes on the same neighbour) carry a localized eigenvector e_i - e_j with
eigenvalue 0 of the normalized adjacency: the columns i and j of H are equal
up to the scale 1/sqrt(d_i) = 1/sqrt(d_j), so H(e_i - e_j) = 0.  A class C of
|C| mutual twins contributes |C| - 1 such eigenvalues.

The paper detects them with a random hash w = Hz (equal w_i = w_j with high
probability means equal neighbourhoods); here the oracle groups nodes by the
exact key "sorted neighbour list" (a dict), so the partition is exact.

Projection: P has as columns the unit vectors of non-motif nodes and the
normalized indicator 1_C/sqrt(|C|) of every class; P P^T z replaces z_i by the
class mean on each class and leaves the other entries.  H_r = P^T H P keeps
the spectrum of H minus the motif eigenvalues, and P P^T commutes with H.

Filtered estimates (reading of the paper, which projects the probes and treats
the removed eigenvalues as known spikes): with z~ = P P^T z,
    mu_m   = (1/(kN)) sum_j z~_j^T T_m(H) z~_j + (sum_C (|C|-1) / N) T_m(0)
    C_im   = (1/k) sum_j z~_ij (T_m(H) z~_j)_i + [i in C] (1 - 1/|C|) T_m(0)
Both stay unbiased: tr(PP^T T_m(H) PP^T) + sum_C (|C|-1) T_m(0) = tr T_m(H),
and the diagonal of (I - PP^T) T_m(H) (I - PP^T) on a class is
(1 - 1/|C|) T_m(0).
"""
from __future__ import annotations

import numpy as np


def twin_classes(g) -> list:
    """Classes of >= 2 nodes with identical open neighbourhoods, in canonical
    order: classes by smallest member, members ascending."""
    groups = {}
    for i in range(g.n):
        key = g.col[g.row_ptr[i]:g.row_ptr[i + 1]].tobytes()
        groups.setdefault(key, []).append(i)
    classes = [sorted(v) for v in groups.values() if len(v) >= 2]
    classes.sort(key=lambda c: c[0])
    return classes


def classes_to_arrays(classes):
    """(class_ptr int64 [n_cls+1], members int32 [N_motif])."""
    ptr = np.zeros(len(classes) + 1, dtype=np.int64)
    for c, members in enumerate(classes):
        ptr[c + 1] = ptr[c] + len(members)
    mem = np.array([i for c in classes for i in c], dtype=np.int32)
    return ptr, mem


def spike_weight(classes, n: int) -> float:
    """Mass of the removed eigenvalue 0 in the DOS: sum_C (|C| - 1) / N."""
    return sum(len(c) - 1 for c in classes) / float(n)


def project(Z: np.ndarray, classes) -> np.ndarray:
    """P P^T Z: each class's rows replaced by their mean."""
    Zr = np.array(Z, dtype=np.float64, copy=True)
    for c in classes:
        idx = np.asarray(c)
        Zr[idx] = Z[idx].mean(axis=0)
    return Zr


def projector_dense(classes, n: int) -> np.ndarray:
    """Dense P P^T (tiny graphs only)."""
    Pm = np.eye(n)
    for c in classes:
        idx = np.asarray(c)
        Pm[np.ix_(idx, idx)] = 1.0 / len(c)
    return Pm


def basis_dense(classes, n: int) -> np.ndarray:
    """Dense orthonormal P [n][r] (tiny graphs only)."""
    in_cls = np.zeros(n, dtype=bool)
    cols = []
    for c in classes:
        v = np.zeros(n)
        v[np.asarray(c)] = 1.0 / np.sqrt(len(c))
        cols.append(v)
        in_cls[np.asarray(c)] = True
    for i in np.flatnonzero(~in_cls):
        v = np.zeros(n)
        v[i] = 1.0
        cols.append(v)
    return np.stack(cols, axis=1) if cols else np.zeros((n, 0))


def filtered_moments(H, Z: np.ndarray, M: int, classes, ldos: bool = True):
    """Filtered estimates as in the module docstring.
    Returns (mu_full [M], mu_smooth [M], mu_pp_smooth [k][M], C [N][M] or None)."""
    from .kpm import stochastic_moments, cheb_at_zero
    n = Z.shape[0]
    Zr = project(Z, classes)
    mu_s, mu_pp, C = stochastic_moments(H, Zr, M, ldos=ldos)
    t0 = cheb_at_zero(M)
    mu_full = mu_s + spike_weight(classes, n) * t0
    if ldos:
        for c in classes:
            C[np.asarray(c), :] += (1.0 - 1.0 / len(c)) * t0[None, :]
    return mu_full, mu_s, mu_pp, C
