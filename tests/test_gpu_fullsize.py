"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (needs an MI355X).

* ER-2000 (20 probes, 100 moments): moments and the 100-bin density, end to end.
* BA-1M + 25k planted twin pairs (64 probes, 500 moments, twin filter, LDOS):
  CSR and twin classes bit-exact; the first 10 global and per-node moments
  against the oracle; exact properties of all 500.
* R-MAT scale 27 (16 probes, 200 moments): sampled rows of the CSR and sampled
  per-node moments against the edge list itself; exact properties.
"""
import numpy as np
import pytest

import synthgraph as sg
from synthgraph.workloads import WORKLOADS
from oracle import graph as og
from oracle import kpm, rng as orng, twins, reconstruct as rc

pytestmark = pytest.mark.gpu


def _z(n, dtype):
    import torch
    return torch.zeros(n, dtype=dtype, device="cuda")


def test_er2000_end_to_end(nd):
    import torch
    W = WORKLOADS["er2000"]
    n, s, d = W.graph(1)
    g = nd.nd_build_csr(n, s, d)
    mu = _z(W.moments, torch.float64)
    nd.nd_cheb_moments(g, None, W.probes, W.moments, 1, 0, mu)
    hist = _z(W.bins, torch.float64)
    nd.nd_reconstruct(mu, 1, W.moments, nd.ND_KERNEL_JACKSON, (), W.bins, -1.0, 1.0, hist)
    g_or = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g_or)
    mu_o, _, _ = kpm.stochastic_moments(H, orng.rademacher(g_or.n, W.probes, 1), W.moments, ldos=False)
    assert np.max(np.abs(mu.cpu().numpy() - mu_o)) < 1e-5
    h_o = rc.histogram(mu_o, W.bins)[0]
    assert np.abs(hist.cpu().numpy() - h_o).sum() < 1e-3
    # against the exact spectrum: the probe estimate is within its statistical error
    mu_x, _ = kpm.exact_moments_eig(H, W.moments)
    assert np.max(np.abs(mu.cpu().numpy() - mu_x)[1:]) < 6.0 * np.sqrt(2.0 / (g_or.n * W.probes))


@pytest.fixture(scope="module")
def ba1m(nd):
    W = WORKLOADS["ba1m_twins"]
    n, s, d = W.graph(1)
    return W, (n, s, d), og.build_csr(n, s, d), nd.nd_build_csr(n, s, d)


def test_ba1m_csr_and_twins_bit_exact(nd, ba1m):
    W, _, g_or, g = ba1m
    ex = nd.nd_graph_export(g)
    assert np.array_equal(ex["row_ptr"], g_or.row_ptr) and np.array_equal(ex["col"], g_or.col)
    assert np.array_equal(ex["old_id"], g_or.old_id)
    assert np.array_equal(ex["dinv_sqrt"].view(np.uint32), g_or.dinv_sqrt.view(np.uint32))
    m = nd.nd_motif_filter(g, 1)
    ptr, mem = nd.nd_motif_export(m)
    p2, m2 = twins.classes_to_arrays(twins.twin_classes(g_or))
    assert np.array_equal(ptr, p2) and np.array_equal(mem, m2)
    assert m.n_classes >= 24_000  # the planted pairs (hub collisions merge a few)


@pytest.mark.parametrize("filtered", [True, False])
def test_ba1m_moments_bench_config(nd, ba1m, filtered):
    import torch
    W, _, g_or, g = ba1m
    k, M, seed, m0 = W.probes, W.moments, 1, 10
    m = nd.nd_motif_filter(g, seed) if filtered else None
    ld = _z(g.n * M, torch.float64)
    mu = _z(M, torch.float64)
    nd.nd_ldos_moments(g, m, k, M, seed, 0, ld, mu=mu)
    C = ld.cpu().numpy().reshape(g.n, M)
    mu = mu.cpu().numpy()
    H = og.normalized_adjacency(g_or)
    Z = orng.rademacher(g_or.n, k, seed)
    if filtered:
        cls = twins.twin_classes(g_or)
        mu_o, _, _, C_o = twins.filtered_moments(H, Z, m0, cls)
        members = np.concatenate([np.asarray(c) for c in cls])
    else:
        mu_o, _, C_o = kpm.stochastic_moments(H, Z, m0)
        members = np.zeros(0, dtype=np.int64)
    assert np.max(np.abs(mu[:m0] - mu_o)) < 1e-5
    assert np.max(np.abs(C[:, :m0] - C_o)) < 1e-5
    # all 500: C_i0 = 1 exactly off the twin classes; global = mean over nodes
    rest = np.ones(g.n, dtype=bool)
    rest[members] = False
    assert np.all(C[rest, 0] == 1.0)
    assert np.max(np.abs(C.mean(axis=0) - mu)) < 1e-9
    # |z~^T T_m(H) z~| <= |z~|^2 since |T_m| <= 1 on the spectrum: the smooth
    # part of every moment is bounded by the smooth mu_0 (the spike adds w T_m(0))
    w = sum(wt for lam, wt in m.spikes) if filtered else 0.0
    t0 = np.cos(np.arange(M) * np.pi / 2).round()
    smooth = mu - w * t0
    assert np.all(np.abs(smooth) <= smooth[0] * (1.0 + 1e-5))


@pytest.fixture(scope="module")
def rmat27(nd):
    import torch
    W = WORKLOADS["rmat27"]
    n, s, d = W.graph(1)
    g = nd.nd_build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    return W, (n, s, d), g


def test_rmat27_sampled_rows_and_moments(nd, rmat27):
    import torch
    W, (n, s, d), g = rmat27
    cid = og.compact_ids_from_edges(n, s, d)
    assert g.n == int(np.sum(cid >= 0))
    old = np.flatnonzero(cid >= 0)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(g.n, 8, replace=False))
    nbs = og.neighbor_sets_from_edges(s, d, old[pick])
    ex = nd.nd_graph_export(g)
    rp, col = ex["row_ptr"], ex["col"]
    assert rp[-1] == g.nnz
    for i in pick:
        assert np.array_equal(old[col[rp[i]:rp[i + 1]]], nbs[int(old[i])])
    del ex, col
    # per-node moment 1: C_i1 = (1/k) sum_j z_ij sum_{v in N(i)} z_vj / sqrt(d_i d_v)
    k, M = W.probes, 3
    ld = _z(g.n * M, torch.float64)
    mu = _z(M, torch.float64)
    nd.nd_ldos_moments(g, None, k, M, 1, 0, ld, mu=mu)
    C = ld.cpu().numpy().reshape(g.n, M)
    nb_all = np.unique(np.concatenate([nbs[int(old[i])] for i in pick]))
    deg_nb = {int(v): a.size for v, a in og.neighbor_sets_from_edges(s, d, nb_all).items()}
    for i in pick:
        N_i = nbs[int(old[i])]
        zi = orng.rademacher_at([i], k, 1)[0]
        zv = orng.rademacher_at(cid[N_i], k, 1)
        dv = np.array([deg_nb[int(v)] for v in N_i], dtype=np.float64)
        hz = (zv / np.sqrt(dv)[:, None]).sum(axis=0) / np.sqrt(N_i.size)
        assert abs(C[i, 1] - np.mean(zi * hz)) < 1e-5
        assert C[i, 0] == 1.0
    assert np.max(np.abs(C.mean(axis=0) - mu.cpu().numpy())) < 1e-9


def test_rmat27_bench_config_properties(nd, rmat27):
    import torch
    W, _, g = rmat27
    mu = _z(W.moments, torch.float64)
    mu_pp = _z(W.probes * W.moments, torch.float64)
    nd.nd_cheb_moments(g, None, W.probes, W.moments, 1, 0, mu, mu_pp)
    mu = mu.cpu().numpy()
    pp = mu_pp.cpu().numpy().reshape(W.probes, W.moments)
    assert np.all(pp[:, 0] == 1.0)
    assert abs(mu[1]) < 1e-3                      # E[mu_1] = tr(H)/N = 0
    assert np.all(np.abs(mu) <= 1.0 + 1e-5)       # |T_m| <= 1 on the spectrum
    # each probe's moments are those of a positive measure: bins of the
    # undamped-free Jackson reconstruction stay non-negative up to fp32 noise
    hist = _z(W.bins, torch.float64)
    nd.nd_reconstruct(mu_pp[: W.moments], 1, W.moments, nd.ND_KERNEL_JACKSON, (), W.bins, -1.0, 1.0, hist)
    h = hist.cpu().numpy()
    assert abs(h.sum() - 1.0) < 1e-9 and h.min() > -1e-4
