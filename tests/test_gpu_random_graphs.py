"""Differential sweep over many small seeded random graphs (self-loops,
duplicate edges, isolated nodes, several components, tiny sizes): every GPU
entry point against the oracle on the same input (needs an MI355X).  fp64
state is used where the oracle's value is exact up to rounding, so the
tolerances are those of fp64 arithmetic."""
import numpy as np
import pytest

from oracle import graph as og
from oracle import kpm, rng as orng, twins, gql

pytestmark = pytest.mark.gpu

ALL_KINDS = {"open", "closed", "pendants", "hubpaths"}


def _random_graph(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 120))
    kind = seed % 4
    if kind == 0:     # sparse random with loops and duplicates
        m = int(rng.integers(1, 3 * n))
        s = rng.integers(0, n, m)
        d = rng.integers(0, n, m)
    elif kind == 1:   # forest-like: attach each node to an earlier one, some left isolated
        s = np.arange(1, n)
        d = np.array([int(rng.integers(0, i)) for i in range(1, n)])
        keep = rng.random(n - 1) < 0.9
        s, d = s[keep], d[keep]
    elif kind == 2:   # dense-ish blocks
        p = float(rng.uniform(0.05, 0.5))
        iu, ju = np.triu_indices(n, 1)
        keep = rng.random(iu.size) < p
        s, d = iu[keep], ju[keep]
    else:             # hub with leaves, pairs and paths
        s, d, nxt = [], [], 1
        while nxt + 2 < n:
            r = int(rng.integers(0, 3))
            if r == 0:
                s += [0]; d += [nxt]; nxt += 1
            elif r == 1:
                s += [0, nxt]; d += [nxt, nxt + 1]; nxt += 2
            else:
                s += [0, nxt, nxt + 1]; d += [nxt, nxt + 1, 1]; nxt += 2
        s, d = np.array(s), np.array(d)
        if s.size == 0:
            s, d = np.array([0]), np.array([1])
    return n, np.asarray(s, np.int32), np.asarray(d, np.int32)


@pytest.mark.parametrize("seed", range(40))
def test_random_graph_against_oracle(nd, seed):
    import torch
    n, s, d = _random_graph(seed)
    g_or = og.build_csr(n, s, d)
    g = nd.nd_build_csr(n, s, d)
    assert g.n == g_or.n and g.nnz == g_or.nnz
    if g.n == 0:
        return
    ex = nd.nd_graph_export(g)
    assert np.array_equal(ex["row_ptr"], g_or.row_ptr) and np.array_equal(ex["col"], g_or.col)
    H = og.normalized_adjacency(g_or)
    f64 = torch.float64
    # motif classes of every kind
    m = nd.nd_motif_filter(g, seed, 0xF)
    ptr, mem = nd.nd_motif_export(m)
    cls, sig = twins.motif_classes(g_or, ALL_KINDS)
    p2, m2 = twins.classes_to_arrays(cls)
    assert np.array_equal(ptr, p2) and np.array_equal(mem, m2)
    assert m.spikes == pytest.approx(twins.spikes(cls, sig, g_or.n), abs=1e-15)
    # moments with fp64 state: plain, filtered, doubling
    k, M = 5, 24
    Z = orng.rademacher(g_or.n, k, seed)
    mu_o, _, C_o = kpm.stochastic_moments(H, Z, M)
    mu = torch.zeros(M, dtype=f64, device="cuda")
    nd.nd_cheb_moments(g, None, k, M, seed, nd.ND_STATE_FP64, mu)
    assert np.max(np.abs(mu.cpu().numpy() - mu_o)) < 1e-10
    nd.nd_cheb_moments(g, None, k, M, seed, nd.ND_STATE_FP64 | nd.ND_MOMENT_DOUBLING, mu)
    assert np.max(np.abs(mu.cpu().numpy() - mu_o)) < 1e-10
    ld = torch.zeros(g.n * M, dtype=f64, device="cuda")
    nd.nd_ldos_moments(g, None, k, M, seed, nd.ND_STATE_FP64, ld)
    assert np.max(np.abs(ld.cpu().numpy().reshape(g.n, M) - C_o)) < 1e-10
    mu_f, mu_s, _, C_f = twins.filtered_moments(H, Z, M, cls, lambdas=sig)
    nd.nd_ldos_moments(g, m, k, M, seed, nd.ND_STATE_FP64, ld, mu=mu)
    assert np.max(np.abs(ld.cpu().numpy().reshape(g.n, M) - C_f)) < 1e-10
    assert np.max(np.abs(mu.cpu().numpy() - mu_f)) < 1e-10
    # exact PDOS: unit probes and nested dissection
    _, l_x = kpm.exact_moments_eig(H, M)
    pd = torch.zeros(g.n * M, dtype=f64, device="cuda")
    nd.nd_pdos_nested(g, M, pd, leaf_size=8)
    assert np.max(np.abs(pd.cpu().numpy().reshape(g.n, M) - l_x)) < 1e-10
    sel = np.arange(g.n, dtype=np.int32)[: 70]
    pu = torch.zeros(sel.size * M, dtype=f64, device="cuda")
    nd.nd_pdos_nodes(g, torch.from_numpy(sel).cuda(), M, nd.ND_STATE_FP64, pu)
    assert np.max(np.abs(pu.cpu().numpy().reshape(sel.size, M) - l_x[sel])) < 1e-10
    # GQL with fp64 vectors: moments of the rules up to degree 2K-1
    K = 6
    nodes = torch.zeros(k * K, dtype=f64, device="cuda")
    weights = torch.zeros(k * K, dtype=f64, device="cuda")
    steps = torch.zeros(k, dtype=torch.int32, device="cuda")
    nd.nd_gql(g, None, k, K, seed, nd.ND_STATE_FP64, nodes, weights, steps)
    nn, ww, ss = (x.cpu().numpy() for x in (nodes, weights, steps))
    rules = [(nn.reshape(k, K)[j, :ss[j]], ww.reshape(k, K)[j, :ss[j]]) for j in range(k)]
    mu_k, _, _ = kpm.stochastic_moments(H, Z, 2 * K, ldos=False)
    assert np.max(np.abs(gql.gql_moments(rules, 2 * K) - mu_k)) < 1e-9
