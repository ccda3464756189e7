"""Pins for the oracle's twin classes, projection, filtered estimates and
density reconstruction (CPU only)."""
import itertools

import numpy as np
import pytest
from scipy import integrate, fft

import synthgraph as sg
from oracle import graph as og
from oracle import kpm, twins, reconstruct as rc


def graph_of(gen):
    n, s, d = gen
    g = og.build_csr(n, s, d)
    return g, og.normalized_adjacency(g)


def brute_twins(g):
    nb = [frozenset(g.neighbors(i).tolist()) for i in range(g.n)]
    seen, classes = set(), []
    for i in range(g.n):
        if i in seen:
            continue
        c = [j for j in range(i, g.n) if nb[j] == nb[i]]
        if len(c) >= 2:
            classes.append(c)
            seen.update(c)
    return classes


@pytest.mark.parametrize("gen", [sg.barabasi_albert(300, 1, seed=2, twin_pairs=20), sg.rmat(9, 4, seed=1),
                                 sg.erdos_renyi(200, 0.008, seed=3)])
def test_twins_match_bruteforce(gen):
    g, _ = graph_of(gen)
    assert twins.twin_classes(g) == brute_twins(g)


def test_twins_textbook():
    g, _ = graph_of(sg.star(6))
    assert twins.twin_classes(g) == [[1, 2, 3, 4, 5, 6]]
    g, _ = graph_of(sg.complete_bipartite(3, 4))
    assert twins.twin_classes(g) == [[0, 1, 2], [3, 4, 5, 6]]
    g, _ = graph_of(sg.cycle(4))
    assert twins.twin_classes(g) == [[0, 2], [1, 3]]
    g, _ = graph_of(sg.complete(5))     # true twins only: open neighbourhoods differ
    assert twins.twin_classes(g) == []


def test_twin_eigenvectors_and_projection_spectrum():
    g, H = graph_of(sg.barabasi_albert(60, 1, seed=5, twin_pairs=6))
    cls = twins.twin_classes(g)
    assert cls
    Hd = H.toarray()
    for c in cls:
        v = np.zeros(g.n)
        v[c[0]], v[c[1]] = 1.0, -1.0
        assert np.allclose(Hd @ v, 0.0, atol=1e-14)   # localized eigenvalue 0
    P = twins.basis_dense(cls, g.n)
    assert np.allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-14)
    lam = np.sort(np.linalg.eigvalsh(Hd))
    lam_r = np.sort(np.linalg.eigvalsh(P.T @ Hd @ P))
    nz = sum(len(c) - 1 for c in cls)
    # removing nz zeros from eig(H) leaves eig(H_r)
    rest = list(lam)
    for _ in range(nz):
        k = int(np.argmin(np.abs(rest)))
        assert abs(rest[k]) < 1e-10
        rest.pop(k)
    assert np.allclose(np.sort(rest), lam_r, atol=1e-10)
    PP = twins.projector_dense(cls, g.n)
    assert np.allclose(PP @ PP, PP) and np.allclose(PP, PP.T)
    assert np.allclose(Hd @ PP, PP @ Hd, atol=1e-14)
    Z = np.random.default_rng(1).normal(size=(g.n, 3))
    assert np.allclose(twins.project(Z, cls), PP @ Z)


def test_filtered_estimates_unbiased_by_enumeration():
    # star + pendant pair graph with twins; all 2^n sign vectors
    n, s, d = 9, np.array([0, 0, 0, 1, 1, 2, 5, 5, 3, 4], np.int32), np.array([1, 2, 3, 4, 5, 6, 7, 8, 6, 6], np.int32)
    g, H = graph_of((n, s, d))
    cls = twins.twin_classes(g)
    assert cls
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=g.n))).T
    M = 10
    mu_full, mu_s, _, C = twins.filtered_moments(H, Z, M, cls)
    mu_x, l_x = kpm.exact_moments_eig(H, M)
    assert np.allclose(mu_full, mu_x, atol=1e-12)
    assert np.allclose(C, l_x, atol=1e-12)
    assert twins.spike_weight(cls, g.n) == sum(len(c) - 1 for c in cls) / g.n


def test_arrays_canonical():
    ptr, mem = twins.classes_to_arrays([[1, 4], [2, 3, 9]])
    assert ptr.tolist() == [0, 2, 5] and mem.tolist() == [1, 4, 2, 3, 9]


# ------------------------------------------------------------ reconstruction
def test_jackson_coefficients():
    g = rc.jackson(100)
    assert g[0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diff(g) < 0)
    assert 0 < g[-1] < 1e-4


def test_jackson_kernel_is_positive():
    # the damped expansion of a point mass at x0 is non-negative (KPM review)
    for x0 in (-0.7, 0.0, 0.33, 1.0):
        M = 64
        mu = np.cos(np.arange(M) * np.arccos(x0))
        x = np.linspace(-0.999, 0.999, 2001)
        assert rc.density(mu, x)[0].min() > -1e-12


def test_bins_equal_quadrature_of_density():
    g_, H = graph_of(sg.erdos_renyi(150, 0.04, seed=2))
    M = 40
    mu, _ = kpm.exact_moments_eig(H, M)
    nb = 16
    h = rc.histogram(mu, nb)[0]
    e = rc.bin_edges(nb, -1, 1)
    for b in range(nb):
        q, _ = integrate.quad(lambda x: rc.density(mu, np.array([x]))[0, 0], e[b], e[b + 1], limit=200)
        assert abs(q - h[b]) < 1e-7
    assert abs(h.sum() - mu[0]) < 1e-13


def test_dct3_equals_direct_sum():
    rng = np.random.default_rng(0)
    mu = rng.normal(size=(3, 30))
    K = 48
    x = rc.cheb_nodes(K)
    direct = rc.density(mu, x) * np.pi * np.sqrt(1 - x * x)[None, :]
    c = mu * rc.jackson(30)[None, :]
    # DCT-III: y_k = x_0 + 2 sum_{m>=1} x_m cos(pi m (k + 1/2) / K)
    pad = np.zeros((3, K))
    pad[:, :30] = c
    via_fft = fft.dct(pad, type=3, axis=1)
    assert np.allclose(direct, via_fft, atol=1e-12)


def test_jackson_error_bound():
    # |int f (rho_M - mu)| <= 6 L / M for Lipschitz f (Sec. 4.1, Jackson's theorem)
    g_, H = graph_of(sg.erdos_renyi(200, 0.05, seed=6))
    lam = np.linalg.eigvalsh(H.toarray())
    f = lambda x: np.abs(x - 0.3)
    for M in (20, 80):
        mu = kpm.cheb_of_eigs(lam, M).mean(axis=1)
        val, _ = integrate.quad(lambda x: f(x) * rc.density(mu, np.array([x]))[0, 0], -1, 1, limit=400, points=[0.3])
        assert abs(val - f(lam).mean()) <= 6.0 / M


def test_exact_moment_histogram_nonnegative_and_spikes():
    g_, H = graph_of(sg.barabasi_albert(200, 1, seed=4, twin_pairs=10))
    mu, _ = kpm.exact_moments_eig(H, 50)
    h = rc.histogram(mu, 50)[0]
    assert h.min() > -1e-12
    h2 = rc.histogram(mu, 50, spikes=[(0.0, 0.25), (1.0, 0.5), (-1.0, 0.125)])[0]
    assert h2[25] - h[25] == pytest.approx(0.25) and h2[49] - h[49] == pytest.approx(0.5)
    assert h2[0] - h[0] == pytest.approx(0.125)
    assert rc.spike_bin(0.0, rc.bin_edges(100, -1, 1)) == 50


def test_exact_histogram_snaps_edges():
    e = rc.exact_histogram(np.array([0.0, 1e-12, -1e-12, 0.5, 1.0]), 4)
    assert np.allclose(e, [0.0, 0.0, 0.6, 0.4], atol=1e-15)


# ------------------------------------------------------------ closed (true) twins
def brute_closed_twins(g):
    nb = [frozenset(g.neighbors(i).tolist()) | {i} for i in range(g.n)]
    seen, classes = set(), []
    for i in range(g.n):
        if i in seen:
            continue
        c = [j for j in range(i, g.n) if nb[j] == nb[i]]
        if len(c) >= 2:
            classes.append(c)
            seen.update(c)
    return classes


def _mixed_graph(seed, n=120, p=0.03, open_pairs=6, closed_pairs=9):
    n0, s, d = sg.erdos_renyi(n, p, seed=seed)
    # dangling pairs (open twins) on random hubs, then adjacent pairs (closed twins)
    rng = np.random.default_rng(seed + 1)
    hubs = rng.choice(n0, open_pairs, replace=False)
    extra_s = np.concatenate([np.arange(n0, n0 + 2 * open_pairs)]).astype(np.int32)
    extra_d = np.repeat(hubs, 2).astype(np.int32)
    s, d = np.concatenate([s, extra_s]), np.concatenate([d, extra_d])
    return sg.plant_adjacent_pairs(n0 + 2 * open_pairs, s, d, closed_pairs, seed + 2)


@pytest.mark.parametrize("gen", [_mixed_graph(1), _mixed_graph(2), sg.friendship(7), sg.complete(6),
                                 sg.rmat(9, 4, seed=4)])
def test_closed_twins_match_bruteforce(gen):
    g, _ = graph_of(gen)
    assert twins.twin_classes(g, "closed") == brute_closed_twins(g)
    # the two kinds never share a node, and "both" is their canonical union
    o, c = twins.twin_classes(g, "open"), twins.twin_classes(g, "closed")
    assert not (set(x for k in o for x in k) & set(x for k in c for x in k))
    assert twins.twin_classes(g, "both") == sorted(o + c, key=lambda k: k[0])


def test_closed_twins_textbook():
    # K_n: every node is a closed twin of every other; H has eigenvalues 1 and
    # -1/(n-1) with multiplicity n-1
    for n in (2, 3, 6):
        g, H = graph_of(sg.complete(n))
        cls = twins.twin_classes(g, "closed")
        assert cls == [list(range(n))]
        assert twins.class_eigenvalue(g, cls[0]) == -1.0 / (n - 1)
        lam = np.sort(np.linalg.eigvalsh(H.toarray()))
        assert np.allclose(lam, [-1.0 / (n - 1)] * (n - 1) + [1.0], atol=1e-13)
    # friendship graph: k blades, each a class of 2 at -1/2
    g, _ = graph_of(sg.friendship(5))
    cls = twins.twin_classes(g, "closed")
    assert cls == [[2 * q + 1, 2 * q + 2] for q in range(5)]
    assert all(twins.class_eigenvalue(g, c) == -0.5 for c in cls)
    assert twins.spikes(cls, [-0.5] * 5, g.n) == [(-0.5, 5 / 11)]
    # open twins have eigenvalue 0; C_4 has only open twins
    g, _ = graph_of(sg.cycle(4))
    assert twins.twin_classes(g, "closed") == []
    assert [twins.class_eigenvalue(g, c) for c in twins.twin_classes(g)] == [0.0, 0.0]


def test_mixed_twins_eigenvectors_and_projection_spectrum():
    g, H = graph_of(_mixed_graph(3))
    cls = twins.twin_classes(g, "both")
    lams = [twins.class_eigenvalue(g, c) for c in cls]
    assert any(l < 0 for l in lams) and any(l == 0 for l in lams)
    Hd = H.toarray()
    for c, lam in zip(cls, lams):
        for j in c[1:]:
            v = np.zeros(g.n)
            v[c[0]], v[j] = 1.0, -1.0
            assert np.allclose(Hd @ v, lam * v, atol=1e-14)
    P = twins.basis_dense(cls, g.n)
    lam_h = list(np.sort(np.linalg.eigvalsh(Hd)))
    lam_r = np.sort(np.linalg.eigvalsh(P.T @ Hd @ P))
    for lam, w in twins.spikes(cls, lams, g.n):
        for _ in range(int(round(w * g.n))):
            k = int(np.argmin(np.abs(np.array(lam_h) - lam)))
            assert abs(lam_h[k] - lam) < 1e-10
            lam_h.pop(k)
    assert np.allclose(np.sort(lam_h), lam_r, atol=1e-10)


def test_filtered_estimates_with_closed_twins_unbiased_by_enumeration():
    # friendship(2) + a dangling pair on the hub + an extra path: open and
    # closed classes; all 2^n sign vectors
    n, s, d = sg.friendship(2)
    s = np.concatenate([s, np.array([0, 0, 1], np.int32)])
    d = np.concatenate([d, np.array([5, 6, 7], np.int32)])
    g, H = graph_of((8, s, d))
    cls = twins.twin_classes(g, "both")
    lams = [twins.class_eigenvalue(g, c) for c in cls]
    assert sorted(lams) == [-0.5, 0.0]
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=g.n))).T
    M = 9
    mu_full, _, _, C = twins.filtered_moments(H, Z, M, cls, lambdas=lams)
    mu_x, l_x = kpm.exact_moments_eig(H, M)
    assert np.allclose(mu_full, mu_x, atol=1e-12)
    assert np.allclose(C, l_x, atol=1e-12)


def test_cheb_at_matches_cosine():
    for lam in (0.0, -0.5, -1.0 / 3.0, 0.9, -1.0, 1.0):
        t = twins.cheb_at(lam, 40)
        assert np.allclose(t, np.cos(np.arange(40) * np.arccos(lam)), atol=1e-12)
    assert twins.cheb_at(0.0, 8).tolist() == [1.0, 0.0, -1.0, 0.0, 1.0, 0.0, -1.0, 0.0]


# ------------------------------------------------------------ the paper's motif figure
def _read_motifs(path):
    blocks, cur = [], None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, *rest = line.split()
        if key == "motif":
            cur = {"name": rest[0], "vector": None, "vector_rw": None}
            blocks.append(cur)
        elif key == "lambda":
            cur["lambda"] = [float(x) for x in rest]
        elif key == "edges":
            cur["edges"] = [tuple(int(v) for v in e.split("-")) for e in rest]
        elif key in ("vector", "vector_rw"):
            cur[key] = {int(a): float(b) for a, b in (x.split(":") for x in rest)}
    return blocks


def test_paper_motif_figure_spikes():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "motif_spikes.txt")
    motifs = _read_motifs(path)
    assert len(motifs) == 6
    for mo in motifs:
        _, hs, hd = sg.complete(5)
        n = 1 + max(max(e) for e in mo["edges"])
        s = np.concatenate([hs, np.array([e[0] for e in mo["edges"]], np.int32)])
        d = np.concatenate([hd, np.array([e[1] for e in mo["edges"]], np.int32)])
        g, H = graph_of((n, s, d))
        Hd = H.toarray()
        lam_all = np.linalg.eigvalsh(Hd)
        for lam in mo["lambda"]:
            assert np.min(np.abs(lam_all - lam)) < 1e-12, (mo["name"], lam)
        v = np.zeros(g.n)
        if mo["vector"]:
            for i, x in mo["vector"].items():
                v[i] = x
        elif mo["vector_rw"]:
            for i, x in mo["vector_rw"].items():
                v[i] = x * np.sqrt(g.deg[i])
        if v.any():
            assert np.allclose(Hd @ v, mo["lambda"][0] * v, atol=1e-13), mo["name"]
    # the two panels that are twin motifs: classes and eigenvalues
    by = {mo["name"]: mo for mo in motifs}
    for name, kind, lam in (("dangling_pair", "open", 0.0), ("triangle_blade", "closed", -0.5)):
        mo = by[name]
        _, hs, hd = sg.complete(5)
        s = np.concatenate([hs, np.array([e[0] for e in mo["edges"]], np.int32)])
        d = np.concatenate([hd, np.array([e[1] for e in mo["edges"]], np.int32)])
        g, _ = graph_of((7, s, d))
        cls = twins.twin_classes(g, kind)
        assert [5, 6] in cls and twins.class_eigenvalue(g, [5, 6]) == lam


# ------------------------------------------------------------ pendant twins
def brute_pendants(g):
    deg = np.diff(g.row_ptr)
    cand = {}
    for b in range(g.n):
        nb = set(g.neighbors(b).tolist())
        leaves = [x for x in nb if deg[x] == 1]
        if deg[b] >= 2 and len(leaves) == 1:
            cand[b] = (leaves[0], frozenset(nb - {leaves[0]}))
    groups = []
    seen = set()
    for b in sorted(cand):
        if b in seen:
            continue
        grp = [c for c in sorted(cand) if cand[c][1] == cand[b][1]]
        seen.update(grp)
        if len(grp) >= 2:
            groups.append((grp, sorted(cand[c][0] for c in grp)))
    return groups


def _pendant_graph(seed):
    # ER core plus groups of 2..4 pendant paths on single core nodes (d = 2)
    # and groups of nodes with a private leaf joined to the same 3 hubs (d = 4)
    n0, s, d = sg.erdos_renyi(80, 0.06, seed=seed)
    rng = np.random.default_rng(seed)
    ss, dd, nxt = list(s), list(d), n0
    for e in rng.choice(n0, 6, replace=False):
        for _ in range(int(rng.integers(2, 5))):
            ss += [int(e), nxt]
            dd += [nxt, nxt + 1]
            nxt += 2
    for _ in range(2):
        hubs = rng.choice(n0, 3, replace=False)
        for _ in range(int(rng.integers(2, 4))):
            ss += [nxt] * 3 + [nxt]
            dd += [int(h) for h in hubs] + [nxt + 1]
            nxt += 2
    return nxt, np.array(ss, np.int32), np.array(dd, np.int32)


@pytest.mark.parametrize("gen", [_pendant_graph(1), _pendant_graph(2), sg.barabasi_albert(400, 1, seed=3)])
def test_pendant_classes_match_bruteforce(gen):
    g, _ = graph_of(gen)
    got = sorted((cb, ca) for cb, ca, _ in twins.pendant_classes(g))
    assert got == sorted((cb, ca) for cb, ca in brute_pendants(g))
    deg = np.diff(g.row_ptr)
    for cb, ca, d in twins.pendant_classes(g):
        assert all(deg[b] == d for b in cb)
    # disjoint from the twin classes
    tw = set(x for k in twins.twin_classes(g, "both") for x in k)
    assert not (tw & set(x for cb, ca, _ in twins.pendant_classes(g) for x in cb + ca))


def test_pendant_spectrum_and_projection():
    """Each group of c pendant twins of degree d removes c-1 eigenvalues at
    +1/sqrt(d) and c-1 at -1/sqrt(d); what is left is the spectrum of P^T H P."""
    g, H = graph_of(_pendant_graph(3))
    cls, sig = twins.motif_classes(g, {"open", "closed", "pendants"})
    Hd = H.toarray()
    lam_h = list(np.sort(np.linalg.eigvalsh(Hd)))
    P = twins.basis_dense(cls, g.n)
    lam_r = np.sort(np.linalg.eigvalsh(P.T @ Hd @ P))
    sp = twins.spikes(cls, sig, g.n)
    for x in (2 ** -0.5, -(2 ** -0.5), 0.5, -0.5):
        assert any(abs(l - x) < 1e-15 for l, _ in sp)
    for lam, w in sp:
        for _ in range(int(round(w * g.n))):
            k = int(np.argmin(np.abs(np.array(lam_h) - lam)))
            assert abs(lam_h[k] - lam) < 1e-10
            lam_h.pop(k)
    assert np.allclose(np.sort(lam_h), lam_r, atol=1e-10)


def test_pendant_filtered_estimates_unbiased_by_enumeration():
    # a hub with three pendant chains and a triangle: 11 nodes, all 2^11 sign vectors
    s = np.array([0, 1, 0, 3, 0, 5, 0, 7, 8, 7, 0], np.int32)
    d = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 9, 10], np.int32)
    g, H = graph_of((11, s, d))
    cls, sig = twins.motif_classes(g, {"open", "closed", "pendants"})
    assert [1, 3, 5] in cls and [2, 4, 6] in cls
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=g.n))).T
    M = 9
    mu_full, _, _, C = twins.filtered_moments(H, Z, M, cls, lambdas=sig)
    mu_x, l_x = kpm.exact_moments_eig(H, M)
    assert np.allclose(mu_full, mu_x, atol=1e-12)
    assert np.allclose(C, l_x, atol=1e-12)


@pytest.mark.parametrize("name,cb", [("two_pendant_paths", [6, 7]), ("pendant_pair_on_three_hubs", [6, 7])])
def test_paper_figure_pendant_panels(name, cb):
    """The figure's panels at +-1/sqrt(2) and (right) +-1/2 are pendant twins."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "motif_spikes.txt")
    mo = [m for m in _read_motifs(path) if m["name"] == name][0]
    _, hs, hd = sg.complete(5)
    s = np.concatenate([hs, np.array([e[0] for e in mo["edges"]], np.int32)])
    d = np.concatenate([hd, np.array([e[1] for e in mo["edges"]], np.int32)])
    g, _ = graph_of((9, s, d))
    cls, sig = twins.motif_classes(g, {"pendants"})
    assert cb in cls and len(cls) == 2
    sp = twins.spikes(cls, sig, g.n)
    assert [l for l, _ in sp] == pytest.approx(sorted(mo["lambda"]), abs=1e-15)
    assert [w for _, w in sp] == [1 / 9, 1 / 9]


# ------------------------------------------------------------ hub paths
def _hub_path_graph(seed):
    # ER core plus groups of 2..4 two-node paths between random pairs of core nodes
    n0, s, d = sg.erdos_renyi(80, 0.08, seed=seed)
    rng = np.random.default_rng(seed)
    ss, dd, nxt = list(s), list(d), n0
    for _ in range(6):
        e, f = (int(x) for x in rng.choice(n0, 2, replace=False))
        for _ in range(int(rng.integers(2, 5))):
            ss += [e, nxt, nxt + 1]
            dd += [nxt, nxt + 1, f]
            nxt += 2
    return nxt, np.array(ss, np.int32), np.array(dd, np.int32)


def brute_hub_paths(g):
    deg = np.diff(g.row_ptr)
    paths = {}
    for x in range(g.n):
        for y in g.neighbors(x).tolist():
            if x < y and deg[x] == 2 and deg[y] == 2:
                e = [u for u in g.neighbors(x).tolist() if u != y][0]
                f = [u for u in g.neighbors(y).tolist() if u != x][0]
                if e != f and deg[e] != 2 and deg[f] != 2:
                    a, b = (x, y) if e < f else (y, x)
                    paths.setdefault((min(e, f), max(e, f)), []).append((a, b))
    return sorted((sorted(a for a, _ in v), sorted(b for _, b in v)) for v in paths.values() if len(v) >= 2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hub_paths_match_bruteforce_and_spectrum(seed):
    g, H = graph_of(_hub_path_graph(seed))
    assert sorted(twins.hub_path_classes(g)) == brute_hub_paths(g)
    cls, sig = twins.motif_classes(g, {"open", "closed", "pendants", "hubpaths"})
    members = [x for c in cls for x in c]
    assert len(members) == len(set(members))      # the kinds never overlap
    Hd = H.toarray()
    lam_h = list(np.sort(np.linalg.eigvalsh(Hd)))
    P = twins.basis_dense(cls, g.n)
    lam_r = np.sort(np.linalg.eigvalsh(P.T @ Hd @ P))
    sp = twins.spikes(cls, sig, g.n)
    assert any(l == 0.5 for l, _ in sp) and any(l == -0.5 for l, _ in sp)
    for lam, w in sp:
        for _ in range(int(round(w * g.n))):
            k = int(np.argmin(np.abs(np.array(lam_h) - lam)))
            assert abs(lam_h[k] - lam) < 1e-10
            lam_h.pop(k)
    assert np.allclose(np.sort(lam_h), lam_r, atol=1e-10)


def test_hub_path_filtered_estimates_unbiased_by_enumeration():
    # three two-node paths between nodes 0 and 1, plus a pendant edge: 9 nodes
    s = np.array([0, 2, 3, 0, 4, 5, 0, 6, 7, 1], np.int32)
    d = np.array([2, 3, 1, 4, 5, 1, 6, 7, 1, 8], np.int32)
    g, H = graph_of((9, s, d))
    cls, sig = twins.motif_classes(g, {"open", "closed", "pendants", "hubpaths"})
    assert [2, 4, 6] in cls and [3, 5, 7] in cls
    Z = np.array(list(itertools.product([-1.0, 1.0], repeat=g.n))).T
    M = 9
    mu_full, _, _, C = twins.filtered_moments(H, Z, M, cls, lambdas=sig)
    mu_x, l_x = kpm.exact_moments_eig(H, M)
    assert np.allclose(mu_full, mu_x, atol=1e-12)
    assert np.allclose(C, l_x, atol=1e-12)


def test_paper_figure_hub_path_panel():
    """The figure's left panel at +-1/2: two paths between the same two hubs."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "motif_spikes.txt")
    mo = [m for m in _read_motifs(path) if m["name"] == "two_paths_between_hubs"][0]
    _, hs, hd = sg.complete(5)
    s = np.concatenate([hs, np.array([e[0] for e in mo["edges"]], np.int32)])
    d = np.concatenate([hd, np.array([e[1] for e in mo["edges"]], np.int32)])
    g, _ = graph_of((9, s, d))
    cls, sig = twins.motif_classes(g, {"hubpaths"})
    assert cls == [[5, 7], [6, 8]]
    sp = twins.spikes(cls, sig, g.n)
    assert [l for l, _ in sp] == sorted(mo["lambda"])
    assert [w for _, w in sp] == [1 / 9, 1 / 9]
