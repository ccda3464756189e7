"""Nested dissection PDOS (Sec. 3.3, Algorithm 1) on the GPU against the
exact PDOS moments of the oracle's eigendecomposition (needs an MI355X).
Graphs with small separators (lattices, trees, rings, paths), graphs
without BFS-level separators (Erdos-Renyi, Barabasi-Albert: multilevel
bisection), disconnected graphs (empty separators), graphs that stay one
dense leaf, and the clean refusal when the blocks would be too large."""
import numpy as np
import pytest

import synthgraph as sg
from oracle import graph as og
from oracle import kpm

pytestmark = pytest.mark.gpu


def _two_grids():
    n1, s1, d1 = sg.grid2d(12, 15)
    n2, s2, d2 = sg.grid2d(9, 9)
    return n1 + n2, np.concatenate([s1, s2 + n1]).astype(np.int32), np.concatenate([d1, d2 + n1]).astype(np.int32)


GRAPHS = {
    "grid": (lambda: sg.grid2d(20, 25), 32),
    "tree": (lambda: sg.barabasi_albert(800, 1, seed=2), 32),
    "ring": (lambda: sg.watts_strogatz(600, 4, 0.02, seed=3), 32),
    "path": (lambda: sg.path(300), 16),
    "cycle": (lambda: sg.cycle(200), 16),
    "two_grids": (_two_grids, 24),
    "star": (lambda: sg.star(150), 32),
    "complete": (lambda: sg.complete(30), 64),
    "er": (lambda: sg.erdos_renyi(300, 0.02, seed=5), 64),
    # no BFS-level separators: split by the multilevel bisection
    "er3000": (lambda: sg.erdos_renyi(3000, 0.004, seed=7), 64),
    "ba3000": (lambda: sg.barabasi_albert(3000, 3, seed=4), 64),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_nested_dissection_pdos_exact(nd, name):
    import torch
    gen, leaf = GRAPHS[name]
    n, s, d = gen()
    g_or = og.build_csr(n, s, d)
    g = nd.nd_build_csr(n, s, d)
    M = 40
    _, l_x = kpm.exact_moments_eig(og.normalized_adjacency(g_or), M)
    pd = torch.zeros(g.n * M, dtype=torch.float64, device="cuda")
    st = nd.nd_pdos_nested(g, M, pd, leaf_size=leaf)
    got = pd.cpu().numpy().reshape(g.n, M)
    assert np.max(np.abs(got - l_x)) < 1e-10, (name, st)
    assert st["tree_nodes"] >= 1 and st["block_entries"] > 0
    if name in ("grid", "tree", "path", "ring"):
        assert st["depth"] >= 2, st
    if name in ("grid", "path", "ring"):
        assert st["separator_nodes"] < g.n // 4, st


def test_nested_dissection_tree_matches_device_call(nd):
    """The statistics nd_pdos_nested reports are those of the host tree
    that nd_nested_tree builds for the same graph and leaf size."""
    import torch
    n, s, d = sg.barabasi_albert(3000, 3, seed=4)
    g_or = og.build_csr(n, s, d)
    g = nd.nd_build_csr(n, s, d)
    pd = torch.zeros(g.n * 3, dtype=torch.float64, device="cuda")
    st = nd.nd_pdos_nested(g, 3, pd, leaf_size=64)
    t = nd.nd_nested_tree(g_or.row_ptr, g_or.col, g_or.n, 64)
    for k in ("tree_nodes", "depth", "separator_nodes", "block_entries"):
        assert st[k] == t[k], (k, st, t)


def test_nested_dissection_refuses_large_blocks(nd):
    import torch
    n, s, d = sg.erdos_renyi(3000, 0.004, seed=7)
    g = nd.nd_build_csr(n, s, d)
    pd = torch.zeros(g.n * 4, dtype=torch.float64, device="cuda")
    with pytest.raises(nd.NDError) as e:
        nd.nd_pdos_nested(g, 4, pd, leaf_size=16, max_entries=100_000)
    assert e.value.status == nd.ND_EUNSUPPORTED
