"""Pins for the large-graph leg of the oracle (oracle/ckpm.c through
oracle/big.py): the plain C graph build and moment recurrence used where the
numpy oracle's intermediate arrays do not fit (CPU only)."""
import numpy as np
import pytest

import synthgraph as sg
from oracle import big, graph as og, kpm, rng as orng
from tests.test_oracle_graph_rng import brute_csr


@pytest.mark.parametrize("seed", range(4))
def test_csr_matches_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 50))
    e = int(rng.integers(0, 150))
    src = rng.integers(0, n, e).astype(np.int32)
    dst = rng.integers(0, n, e).astype(np.int32)
    src = np.concatenate([src, dst[: e // 3], src[: e // 5]])   # duplicates, both orientations, loops
    dst = np.concatenate([dst, src[: e // 3], src[: e // 5]])
    old, rows = brute_csr(n, src, dst)
    if not old:
        with pytest.raises(ValueError):
            big.BigGraph(n, src, dst).moments(1, 1)
        return
    g = big.BigGraph(n, src, dst)
    assert g.n == len(old) and g.old_id().tolist() == old
    rp, col = g.row_ptr(), g.col_view()
    for i, r in enumerate(rows):
        assert col[rp[i]:rp[i + 1]].tolist() == r


@pytest.mark.parametrize("make", [lambda: sg.rmat(11, 8, seed=3), lambda: sg.barabasi_albert(1500, 3, seed=2, twin_pairs=40),
                                  lambda: sg.watts_strogatz(800, 4, 0.3, seed=1)])
def test_unit_probes_give_exact_pdos(make):
    """Unit probes e_v give T_m(H)_vv exactly: against a dense
    eigendecomposition (eqn pdoscoeff)."""
    n, s, d = make()
    g = big.BigGraph(n, s, d)
    g_or = og.build_csr(n, s, d)
    _, ldos = kpm.exact_moments_eig(og.normalized_adjacency(g_or), 40)
    nodes = np.array([0, 1, g.n // 2, g.n - 1, int(np.argmax(g_or.deg))])
    pp, _ = g.moments(0, 40, unit_nodes=nodes)
    assert np.max(np.abs(pp - ldos[nodes])) < 1e-12


def test_probes_and_moments_match_numpy_oracle():
    """Same Rademacher probes (the published SplitMix64 construction, pinned
    in the numpy oracle's tests) and the same estimates."""
    n, s, d = sg.rmat(12, 8, seed=7)
    g = big.BigGraph(n, s, d)
    g_or = og.build_csr(n, s, d)
    Z = orng.rademacher(g_or.n, 9, 77)
    mu, pp, C = kpm.stochastic_moments(og.normalized_adjacency(g_or), Z, 25)
    rows = np.array([0, 3, 100, g.n - 1])
    pp2, ld2 = g.moments(9, 25, seed=77, rows=rows)
    assert np.max(np.abs(pp2 - pp)) < 1e-12
    assert np.max(np.abs(ld2 - C[rows])) < 1e-12
    assert np.all(pp2[:, 0] == 1.0)


def test_closed_forms():
    """mu_0 = 1 exactly for Rademacher probes; the second Chebyshev moment of
    each node row is 2 sum_j A_ij/(d_i d_j) - 1 in expectation -- exact for
    the unit-probe diagonal; odd moments of a bipartite graph vanish for
    unit probes."""
    n, s, d = sg.grid2d(12, 9)                 # bipartite
    g = big.BigGraph(n, s, d)
    g_or = og.build_csr(n, s, d)
    pp = np.concatenate([g.moments(0, 9, unit_nodes=np.arange(a, min(a + 64, g.n)))[0] for a in range(0, g.n, 64)])
    assert np.allclose(pp[:, 2], kpm.cheb_moment_2_diag(g_or), atol=1e-13)
    assert np.max(np.abs(pp[:, 1::2])) < 1e-13
    pr, _ = g.moments(5, 3, seed=1)
    assert np.all(pr[:, 0] == 1.0)


def test_bad_arguments():
    with pytest.raises(ValueError):
        big.BigGraph(3, np.array([0, 5], np.int32), np.array([1, 1], np.int32))
    g = big.BigGraph(4, np.array([0, 1, 2], np.int32), np.array([1, 2, 3], np.int32))
    with pytest.raises(ValueError):
        g.moments(65, 3)
    with pytest.raises(ValueError):
        g.moments(1, 3, rows=[7])
