"""Pins for the oracle's graph builder and probe generator (CPU only)."""
import numpy as np
import pytest

import synthgraph as sg
from oracle import graph as og
from oracle import rng as orng


def brute_csr(n_nodes, src, dst):
    nb = {}
    for a, b in zip(src.tolist(), dst.tolist()):
        if a == b:
            continue
        nb.setdefault(a, set()).add(b)
        nb.setdefault(b, set()).add(a)
    old = sorted(nb)
    new = {o: i for i, o in enumerate(old)}
    rows = [sorted(new[v] for v in nb[o]) for o in old]
    return old, rows


@pytest.mark.parametrize("seed", range(6))
def test_csr_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    e = int(rng.integers(0, 120))
    src = rng.integers(0, n, e).astype(np.int32)
    dst = rng.integers(0, n, e).astype(np.int32)
    # duplicates (both orientations) and self-loops on purpose
    src = np.concatenate([src, dst[: e // 3], src[: e // 4]])
    dst = np.concatenate([dst, src[: e // 3], src[: e // 4]])
    g = og.build_csr(n, src, dst)
    old, rows = brute_csr(n, src, dst)
    assert g.old_id.tolist() == old
    assert g.n == len(old)
    for i, r in enumerate(rows):
        assert g.neighbors(i).tolist() == r
        assert g.deg[i] == len(r)
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.nnz == sum(len(r) for r in rows)


def test_csr_invariants_rmat():
    n, s, d = sg.rmat(12, 8, seed=3)
    g = og.build_csr(n, s, d)
    A = og.normalized_adjacency(g)
    assert (A != A.T).nnz == 0                             # symmetric
    assert np.all(g.deg > 0)                               # isolated dropped
    assert np.all(np.diff(g.old_id) > 0)                   # monotone relabel
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert not np.any(rows == g.col)                       # no self-loops
    same = rows[1:] == rows[:-1]
    assert np.all(g.col[1:][same] > g.col[:-1][same])      # sorted, no duplicates
    assert g.deg.sum() == g.nnz


def test_csr_empty_and_isolated():
    g = og.build_csr(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert g.n == 0 and g.nnz == 0 and g.row_ptr.tolist() == [0]
    g = og.build_csr(5, np.array([2, 3], np.int32), np.array([2, 3], np.int32))  # only loops
    assert g.n == 0
    with pytest.raises(ValueError):
        og.build_csr(3, np.array([0], np.int32), np.array([3], np.int32))


def test_dinv_sqrt_rounding():
    # perfect powers of 4: 1/sqrt(4^k) = 2^-k exactly
    deg = np.array([4**k for k in range(12)], np.int64)
    n = len(deg)
    g = og.Graph(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), deg,
                 np.arange(n, dtype=np.int32), (1.0 / np.sqrt(deg.astype(np.float64))).astype(np.float32))
    assert np.array_equal(g.dinv_sqrt, np.array([2.0**-k for k in range(12)], np.float32))
    # the stored value is the fp32 nearest to the real 1/sqrt(d): compare with
    # its fp32 neighbours using exact rational arithmetic on d * x^2 - 1
    _, s, d = sg.rmat(10, 16, seed=1)
    g = og.build_csr(1024, s, d)
    from fractions import Fraction
    for di, x in zip(g.deg[:300].tolist(), g.dinv_sqrt[:300].tolist()):
        # x is the fp32 nearest 1/sqrt(d) iff 1/sqrt(d) lies between the
        # midpoints to its fp32 neighbours: m_lo^2 d <= 1 <= m_hi^2 d, exactly
        lo = Fraction(float(np.nextafter(np.float32(x), np.float32(0))))
        hi = Fraction(float(np.nextafter(np.float32(x), np.float32(2))))
        fx = Fraction(x)
        m_lo, m_hi = (fx + lo) / 2, (fx + hi) / 2
        assert m_lo * m_lo * di <= 1 <= m_hi * m_hi * di


def test_perron_vector():
    # D^{1/2} 1 is an eigenvector of D^{-1/2} A D^{-1/2} with eigenvalue 1
    n, s, d = sg.erdos_renyi(300, 0.03, seed=2)
    g = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g)
    v = np.sqrt(g.deg.astype(np.float64))
    assert np.allclose(H @ v, v, atol=1e-12)


def test_neighbor_sets_from_edges():
    n, s, d = sg.rmat(10, 8, seed=4)
    g = og.build_csr(n, s, d)
    pick = g.old_id[[0, 5, 17, g.n - 1]]
    nbs = og.neighbor_sets_from_edges(s, d, pick)
    for o in pick:
        i = int(np.searchsorted(g.old_id, o))
        assert nbs[int(o)].tolist() == g.old_id[g.neighbors(i)].tolist()


# ---------------------------------------------------------------- probes
def test_splitmix64_published_vector():
    # the first outputs of SplitMix64 seeded with 1234567, as printed with the
    # reference implementation's test vector
    assert [orng.splitmix64(1234567, n) for n in range(1, 6)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    v = orng.splitmix64_np(1234567, np.arange(1, 6, dtype=np.uint64))
    assert v.tolist() == [orng.splitmix64(1234567, n) for n in range(1, 6)]


def test_rademacher_stats():
    Z = orng.rademacher(20000, 8, seed=11)
    assert set(np.unique(Z).tolist()) == {-1.0, 1.0}
    # mean 0, variance 1, probes uncorrelated: 5 sigma bounds
    assert np.all(np.abs(Z.mean(axis=0)) < 5 / np.sqrt(20000))
    C = (Z.T @ Z) / 20000
    off = C[~np.eye(8, dtype=bool)]
    assert np.all(np.abs(off) < 5 / np.sqrt(20000))
    # definition: the sign is the top bit of output i+1 of probe j's stream
    key = orng.probe_key(11, 3)
    assert Z[7, 3] == (-1.0 if orng.splitmix64(key, 8) >> 63 else 1.0)


def test_gaussian_stats():
    from scipy import stats
    Z = orng.gaussian(50000, 2, seed=5)
    for j in range(2):
        assert stats.kstest(Z[:, j], "norm").pvalue > 1e-4
    assert abs(Z.var() - 1.0) < 0.02
    assert np.array_equal(Z, Z.astype(np.float32).astype(np.float64))


def test_rademacher_at_and_compact_ids():
    Z = orng.rademacher(300, 5, seed=9)
    pick = np.array([0, 17, 299, 5])
    assert np.array_equal(orng.rademacher_at(pick, 5, 9), Z[pick])
    n, s, d = sg.rmat(11, 4, seed=2)
    g = og.build_csr(n, s, d)
    cid = og.compact_ids_from_edges(n, s, d)
    assert np.array_equal(cid[g.old_id], np.arange(g.n))
    assert np.sum(cid >= 0) == g.n
