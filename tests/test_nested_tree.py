"""The nested-dissection tree (Sec. 3.3, Algorithm 1's partition step) built
on the host by the library, checked on the CPU: every node sits in exactly
one separator or leaf, the tree is a tree, and every edge joins two nodes
whose owners lie on one root-to-leaf path -- the property the block
recurrence (eqn ndchebsep) needs.  Graphs without BFS-level separators
(Erdos-Renyi, Barabasi-Albert) are split by the multilevel bisection."""
import numpy as np
import pytest

import synthgraph as sg
from oracle import graph as og


def _two_grids():
    n1, s1, d1 = sg.grid2d(12, 15)
    n2, s2, d2 = sg.grid2d(9, 9)
    return n1 + n2, np.concatenate([s1, s2 + n1]).astype(np.int32), np.concatenate([d1, d2 + n1]).astype(np.int32)


GRAPHS = {
    "grid": (lambda: sg.grid2d(40, 50), 32),
    "tree": (lambda: sg.barabasi_albert(3000, 1, seed=2), 32),
    "ring": (lambda: sg.watts_strogatz(2000, 4, 0.02, seed=3), 32),
    "path": (lambda: sg.path(500), 16),
    "two_grids": (_two_grids, 24),
    "star": (lambda: sg.star(150), 32),
    "complete": (lambda: sg.complete(60), 16),
    "er3000": (lambda: sg.erdos_renyi(3000, 0.004, seed=7), 64),
    "ba3000": (lambda: sg.barabasi_albert(3000, 3, seed=4), 64),
    "er20000": (lambda: sg.erdos_renyi(20000, 6.0 / 20000, seed=5), 64),
}


def _depths(parent):
    dep = np.zeros(parent.size, np.int64)
    for t in range(parent.size):
        dep[t] = 0 if parent[t] < 0 else dep[parent[t]] + 1
    return dep


def _is_ancestor(parent, dep, a, b):
    """a is b or an ancestor of b."""
    while dep[b] > dep[a]:
        b = parent[b]
    return a == b


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_nested_tree_separates(nd_host, name):
    nd = nd_host
    gen, leaf = GRAPHS[name]
    n, s, d = gen()
    g = og.build_csr(n, s, d)
    t = nd.nd_nested_tree(g.row_ptr, g.col, g.n, leaf)
    owner, parent = t["owner"], t["parent"]
    T = t["tree_nodes"]
    assert np.all(owner >= 0) and np.all(owner < T)
    assert parent[0] == -1 and np.all(parent[1:] >= 0) and np.all(parent[1:] < np.arange(1, T))
    dep = _depths(parent)
    assert int(dep.max()) == t["depth"]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    ou, ov = owner[rows], owner[g.col]
    # each edge: one owner is an ancestor of (or equal to) the other
    for a, b in set(zip(ou.tolist(), ov.tolist())):
        assert _is_ancestor(parent, dep, a, b) or _is_ancestor(parent, dep, b, a), (name, a, b)
    if name in ("grid", "path", "ring", "tree"):
        assert t["separator_nodes"] < g.n // 3, t
    if name.startswith(("er", "ba")):
        assert t["depth"] >= 3, t


def test_multilevel_separators_are_small_on_random_graphs(nd_host):
    nd = nd_host
    """On an Erdos-Renyi graph of mean degree 6 the largest separator stays
    a modest fraction of the nodes and the block entries fit a few hundred
    MB."""
    n, s, d = sg.erdos_renyi(20000, 6.0 / 20000, seed=5)
    g = og.build_csr(n, s, d)
    t = nd.nd_nested_tree(g.row_ptr, g.col, g.n, 64)
    T = t["tree_nodes"]
    internal = np.zeros(T, bool)
    internal[t["parent"][1:]] = True
    sizes = np.bincount(t["owner"], minlength=T)
    largest = int(sizes[internal].max())
    assert 0 < largest < 0.35 * g.n, largest       # measured: 0.32 n
    assert t["block_entries"] < 2e8, t


def test_nested_tree_errors(nd_host):
    nd = nd_host
    g = og.build_csr(*sg.path(10))
    with pytest.raises(nd.NDError):
        nd.nd_nested_tree(g.row_ptr, g.col, g.n, 0)
    bad = g.col.copy()
    bad[0] = 99
    with pytest.raises(nd.NDError):
        nd.nd_nested_tree(g.row_ptr, bad, g.n, 4)
    rp = g.row_ptr.copy()
    rp[3], rp[4] = rp[4], rp[3]
    with pytest.raises(nd.NDError):
        nd.nd_nested_tree(rp, g.col, g.n, 4)
