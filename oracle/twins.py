"""Twin motifs and probe projection (Sec. 3.4, motif filtering, and the
motif figure there that lists the spectral signature of each motif).

Oracle: test infrastructure only (tests, the smoke check and the CPU baseline
of the benchmark use it; the GPU library never does).

Two nodes with identical open neighbourhoods ("node copies", e.g. two dangling
nodes on the same neighbour) carry a localized eigenvector e_i - e_j with
eigenvalue 0 of the normalized adjacency: the columns i and j of H are equal
up to the scale 1/sqrt(d_i) = 1/sqrt(d_j), so H(e_i - e_j) = 0.  A class C of
|C| mutual twins contributes |C| - 1 such eigenvalues.

Two adjacent nodes with identical closed neighbourhoods N[i] = N(i) + {i}
(e.g. the two blade nodes of a triangle hanging off a hub) have equal degree
d and A(e_i - e_j) = e_j - e_i, so H(e_i - e_j) = -(1/d)(e_i - e_j): a class
C of such nodes contributes |C| - 1 eigenvalues at -1/d (the spikes at -1/2,
-1/3, ... of the paper's spectra).  A node cannot have twins of both kinds
(an open twin j and a closed twin k would force k ~ j, hence j in N[i]).

Pendant twins (the figure's panels at +-1/sqrt(2) and, on the right, +-1/2):
c >= 2 nodes B of degree d >= 2 that each carry one private leaf A (and no
other leaf) and have the same remaining neighbourhood N(B) - {A}.  On the
differences between copies H couples each A to its B with h = 1/sqrt(d) and
the shared neighbours cancel, so the 2(c - 1)-dimensional space of
differences carries c - 1 eigenvalues at +h and c - 1 at -h (d = 2: pendant
chains E - B - A on one node E, +-1/sqrt(2); d = 4: a pendant edge on nodes
joined to the same three hubs, +-1/2).  They are handled as two classes (the
A's and the B's) whose projection is again the class mean; each class holds
half of the pair, written as the signature [(+h, 1/2), (-h, 1/2)], and the
diagonal of T_m(H) on the removed space is (1 - 1/c)(T_m(h) + T_m(-h))/2.
Pendant-twin nodes are never twins of either kind.

Hub paths (the figure's left panel at +-1/2): c >= 2 paths E - X - Y - F
between the same two distinct nodes E, F, with X and Y of degree 2 and no
other degree-2 neighbour (so the path has exactly two interior nodes).  On
the differences between copies H couples each X to its Y with 1/2, so the
X's and the Y's form two classes holding c - 1 eigenvalues at +1/2 and c - 1
at -1/2, with the same paired signature as pendant twins.  The X side is the
one adjacent to the smaller of the two end nodes.  These nodes are never
twins or pendant twins.

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


def twin_classes(g, kind: str = "open") -> list:
    """Classes of >= 2 nodes with identical open neighbourhoods (kind
    "open"), identical closed neighbourhoods ("closed"), or both kinds
    ("both"; the two never share a node), in canonical order: classes by
    smallest member, members ascending."""
    if kind == "both":
        classes = twin_classes(g, "open") + twin_classes(g, "closed")
        classes.sort(key=lambda c: c[0])
        return classes
    if kind not in ("open", "closed"):
        raise ValueError(kind)
    groups = {}
    for i in range(g.n):
        nb = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        key = tuple(sorted(nb.tolist() + [i])) if kind == "closed" else nb.tobytes()
        groups.setdefault(key, []).append(i)
    classes = [sorted(v) for v in groups.values() if len(v) >= 2]
    classes.sort(key=lambda c: c[0])
    return classes


def class_eigenvalue(g, cls) -> float:
    """The eigenvalue of H on the differences inside a class: 0 for open
    twins (members not adjacent), -1/d for closed twins (members adjacent,
    common degree d)."""
    a, b = cls[0], cls[1]
    nb = g.col[g.row_ptr[a]:g.row_ptr[a + 1]]
    if b in set(nb.tolist()):
        return -1.0 / float(nb.size)
    return 0.0


def signature(sig):
    """A class's removed eigenvalues as [(lambda, fraction)]: a plain number is
    one eigenvalue taking all |C| - 1 removed dimensions."""
    if isinstance(sig, (int, float, np.floating)):
        return [(float(sig), 1.0)]
    return [(float(l), float(f)) for l, f in sig]


def pendant_classes(g) -> list:
    """Pendant twins: triples (B-class, A-class, d), members ascending, for
    every group of >= 2 nodes B (degree d >= 2, exactly one leaf neighbour A)
    with equal N(B) - {A}."""
    deg = np.diff(g.row_ptr)
    groups = {}
    for b in range(g.n):
        if deg[b] < 2:
            continue
        nb = g.neighbors(b).tolist()
        leaves = [x for x in nb if deg[x] == 1]
        if len(leaves) != 1:
            continue
        rest = tuple(x for x in nb if x != leaves[0])
        groups.setdefault(rest, []).append((b, leaves[0]))
    out = []
    for rest, v in groups.items():
        if len(v) >= 2:
            out.append((sorted(b for b, _ in v), sorted(a for _, a in v), len(rest) + 1))
    out.sort(key=lambda t: min(t[0][0], t[1][0]))
    return out


def hub_path_classes(g) -> list:
    """Hub paths: pairs (X-class, Y-class), members ascending, for every pair
    of end nodes E < F joined by >= 2 paths E - X - Y - F (deg X = deg Y = 2,
    X's and Y's other neighbours not of degree 2, E != F)."""
    deg = np.diff(g.row_ptr)
    groups = {}
    for x in range(g.n):
        if deg[x] != 2:
            continue
        nb = g.neighbors(x).tolist()
        two = [u for u in nb if deg[u] == 2]
        if len(two) != 1:
            continue
        y = two[0]
        e = nb[0] if nb[1] == y else nb[1]
        ynb = g.neighbors(y).tolist()
        f = ynb[0] if ynb[1] == x else ynb[1]
        if deg[f] == 2 or e == f:
            continue
        if e < f:
            groups.setdefault((e, f), ([], []))[0].append(x)
        else:
            groups.setdefault((f, e), ([], []))[1].append(x)
    out = []
    for key in sorted(groups):
        xs, ys = groups[key]
        if len(xs) >= 2:
            out.append((sorted(xs), sorted(ys)))
    return out


def motif_classes(g, kinds) -> tuple:
    """All classes of the requested kinds ("open", "closed", "pendants",
    "hubpaths"), in canonical order (by smallest member), with their
    signatures."""
    cls = []
    for kind in ("open", "closed"):
        if kind in kinds:
            cls += [(c, class_eigenvalue(g, c)) for c in twin_classes(g, kind)]
    if "pendants" in kinds:
        for cb, ca, d in pendant_classes(g):
            h = float(np.sqrt(1.0 / d))   # 1/sqrt(d), correctly rounded
            cls += [(cb, [(h, 0.5), (-h, 0.5)]), (ca, [(h, 0.5), (-h, 0.5)])]
    if "hubpaths" in kinds:
        for cx, cy in hub_path_classes(g):
            cls += [(cx, [(0.5, 0.5), (-0.5, 0.5)]), (cy, [(0.5, 0.5), (-0.5, 0.5)])]
    cls.sort(key=lambda t: t[0][0])
    return [c for c, _ in cls], [sgn for _, sgn in cls]


def spikes(classes, lambdas, n: int) -> list:
    """Point masses removed from the DOS: [(lambda, sum over classes of
    (|C| - 1) times the class's share of that eigenvalue / N)], ascending."""
    acc = {}
    for c, sig in zip(classes, lambdas):
        for lam, f in signature(sig):
            acc[lam] = acc.get(lam, 0.0) + (len(c) - 1) * f
    return [(lam, acc[lam] / float(n)) for lam in sorted(acc)]


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


def cheb_at(lam: float, M: int) -> np.ndarray:
    """T_m(lambda), m = 0..M-1, by the three-term recurrence (exact
    {1, 0, -1, 0, ...} at lambda = 0)."""
    t = np.zeros(M)
    if M > 0:
        t[0] = 1.0
    if M > 1:
        t[1] = lam
    for m in range(1, M - 1):
        t[m + 1] = 2.0 * lam * t[m] - t[m - 1]
    return t


def filtered_moments(H, Z: np.ndarray, M: int, classes, ldos: bool = True, lambdas=None):
    """Filtered estimates as in the module docstring, for classes whose
    removed eigenvalues are `lambdas` (signatures; all 0, open twins, when
    omitted):
        mu_m = smooth part + sum_C (|C|-1)/N sum_s f_s T_m(lambda_s)
        C_im = smooth part + [i in C] (1 - 1/|C|) sum_s f_s T_m(lambda_s).
    Returns (mu_full [M], mu_smooth [M], mu_pp_smooth [k][M], C [N][M] or None)."""
    from .kpm import stochastic_moments
    n = Z.shape[0]
    if lambdas is None:
        lambdas = [0.0] * len(classes)
    Zr = project(Z, classes)
    mu_s, mu_pp, C = stochastic_moments(H, Zr, M, ldos=ldos)
    mu_full = np.array(mu_s, copy=True)
    for lam, w in spikes(classes, lambdas, n):
        mu_full += w * cheb_at(lam, M)
    if ldos:
        for c, sig in zip(classes, lambdas):
            t = sum(f * cheb_at(lam, M) for lam, f in signature(sig))
            C[np.asarray(c), :] += (1.0 - 1.0 / len(c)) * t[None, :]
    return mu_full, mu_s, mu_pp, C
