"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (needs an MI355X).

* ER-2000 (20 probes, 100 moments): moments and the 100-bin density, end to end.
* BA-1M + 25k planted twin pairs (64 probes, 500 moments, twin filter, LDOS):
  CSR and twin classes bit-exact; the first 10 global and per-node moments
  against the oracle run here; all 500 per-probe global moments and the
  per-node moments of 192 nodes (hubs, twin members, others), filter on and
  off, against the oracle's stored values (tests/golden/make_goldens.py),
  and the 100-bin Jackson density of those moments and the 50-bin PDOS of
  each stored node within 1e-3 L1; exact properties of all 500.
* R-MAT scale 27 (16 probes, 200 moments): sampled rows of the CSR and sampled
  per-node moments against the edge list itself; all 200 per-probe global
  moments and the per-node moments of 64 nodes (among them the 16 largest
  rows, which the device splits across wavefronts) against the oracle's
  stored values, and their 100-bin density and the stored nodes' 50-bin
  PDOS within 1e-3 L1; exact properties.
* R-MAT scale 22 ef 16 (32 probes, 1000 moments; the precision study): every
  per-probe global moment and the per-node moments of 128 nodes in fp32 and
  fp64 state, and the 200-bin density, against the oracle's stored values.

fp32 bars: 1e-5 for m <= 200 (global and per-node); beyond, the envelope
C_LIN m 2^-24 (the row update is fp64, so the per-node error grows about
linearly; C_LIN is three times the largest err / (m 2^-24) measured on these
workloads).
"""
import os

import numpy as np
import pytest

import synthgraph as sg
from synthgraph.workloads import WORKLOADS
from oracle import graph as og
from oracle import kpm, rng as orng, twins, reconstruct as rc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS32 = 2.0 ** -24
C_LIN = 1.3


def _golden(name):
    return np.load(os.path.join(GOLDEN, name), allow_pickle=False)


def _fp32_envelope(M):
    """Allowed |error| of fp32-state moments m = 0..M-1 (see the module docstring)."""
    m = np.arange(M, dtype=np.float64)
    return np.where(m <= 200, 1e-5, np.maximum(1e-5, C_LIN * m * EPS32))


def _check_envelope(err, M, what):
    """err [..., M]: max over leading axes within the envelope of each m."""
    e = np.asarray(err).reshape(-1, M).max(axis=0)
    env = _fp32_envelope(M)
    bad = np.flatnonzero(e > env)
    assert bad.size == 0, "%s: m=%d err %.3e > %.3e (max over m<=200: %.3e)" % (
        what, int(bad[0]), float(e[bad[0]]), float(env[bad[0]]), float(e[:201].max()))


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
    # bit-identical on a second run of the same configuration (fixed-order
    # sums, split rows included)
    mu_pp2 = _z(W.probes * W.moments, torch.float64)
    nd.nd_cheb_moments(g, None, W.probes, W.moments, 1, 0, _z(W.moments, torch.float64), mu_pp2)
    assert torch.equal(mu_pp, mu_pp2)


@pytest.mark.parametrize("filtered", [False, True])
def test_ba1m_all_moments_vs_oracle_goldens(nd, ba1m, filtered):
    """All 500 moments of the benchmark configuration: per-probe global
    moments (smooth part when filtering) and the per-node moments of the
    stored nodes, against the fp64 oracle (Sec. 3.1 eqn doscoeff / eqn
    pdoscoeff; Sec. 3.4 for the filter)."""
    import torch
    W, _, g_or, g = ba1m
    G = _golden("ba1m_twins_oracle.npz")
    k, M, seed = W.probes, W.moments, int(G["probe_seed"])
    assert g.n == int(G["n"]) and g.nnz == int(G["nnz"])
    m = nd.nd_motif_filter(g, seed) if filtered else None
    mu = _z(M, torch.float64)
    pp = _z(k * M, torch.float64)
    nd.nd_cheb_moments(g, m, k, M, seed, 0, mu, pp)
    pp = pp.cpu().numpy().reshape(k, M)
    want_pp = G["mu_pp_smooth"] if filtered else G["mu_pp_plain"]
    _check_envelope(np.abs(pp - want_pp), M, "BA-1M per-probe moments")
    # the Jackson density of the (smooth, when filtering) global moments
    # (Sec. 4.1): device reconstruction of the device moments against the
    # oracle's reconstruction of its own
    hist = _z(W.bins, torch.float64)
    nd.nd_reconstruct(mu, 1, M, nd.ND_KERNEL_JACKSON, (), W.bins, -1.0, 1.0, hist)
    l1 = float(np.abs(hist.cpu().numpy() - rc.histogram(want_pp.mean(axis=0), W.bins)[0]).sum())
    assert l1 < 1e-3, l1
    ld = _z(g.n * M, torch.float64)
    mu2 = _z(M, torch.float64)
    nd.nd_ldos_moments(g, m, k, M, seed, 0, ld, mu=mu2)
    nodes = G["nodes"]
    C_dev = ld.view(g.n, M)[torch.from_numpy(nodes).cuda()].contiguous()
    C = C_dev.cpu().numpy()
    want_C = G["ldos_filtered"] if filtered else G["ldos_plain"]
    _check_envelope(np.abs(C - want_C), M, "BA-1M per-node moments")
    # the benchmark's per-node 50-bin PDOS histograms of these rows, each
    # within 1e-3 L1 of the oracle's reconstruction of its own moments
    pd = _z(nodes.size * 50, torch.float64)
    nd.nd_reconstruct(C_dev, nodes.size, M, nd.ND_KERNEL_JACKSON, (), 50, -1.0, 1.0, pd)
    l1 = np.abs(pd.cpu().numpy().reshape(nodes.size, 50) - rc.histogram(want_C, 50)).sum(axis=1)
    assert l1.max() < 1e-3, ("per-node 50-bin PDOS L1", float(l1.max()), int(nodes[l1.argmax()]))
    if filtered:
        _check_envelope(np.abs(mu2.cpu().numpy() - G["mu_full_filtered"]), M, "BA-1M filtered full moments")


def test_rmat27_all_moments_vs_oracle_goldens(nd, rmat27):
    """R-MAT-27, all 200 moments of the benchmark configuration: per-probe
    global moments and per-node moments of the stored nodes (the 16 largest
    rows, split into chunks on the device, and 48 others) against the
    oracle's C leg (Sec. 3.1 eqn doscoeff / eqn pdoscoeff)."""
    import torch
    W, _, g = rmat27
    G = _golden("rmat27_oracle.npz")
    k, M, seed = W.probes, G["mu_pp"].shape[1], int(G["probe_seed"])
    assert g.n == int(G["n"]) and g.nnz == int(G["nnz"])
    ex = nd.nd_graph_export(g)
    nodes = G["nodes"]
    assert np.array_equal(np.diff(ex["row_ptr"])[nodes], G["node_degree"])
    del ex
    mu = _z(M, torch.float64)
    pp = _z(k * M, torch.float64)
    nd.nd_cheb_moments(g, None, k, M, seed, 0, mu, pp)
    e = np.abs(pp.cpu().numpy().reshape(k, M) - G["mu_pp"])
    assert e.max() < 1e-5, ("per-probe", float(e.max()), np.unravel_index(e.argmax(), e.shape))
    hist = _z(W.bins, torch.float64)
    nd.nd_reconstruct(mu, 1, M, nd.ND_KERNEL_JACKSON, (), W.bins, -1.0, 1.0, hist)
    l1 = float(np.abs(hist.cpu().numpy() - rc.histogram(G["mu_pp"].mean(axis=0), W.bins)[0]).sum())
    assert l1 < 1e-3, ("100-bin density L1", l1)
    ld = _z(g.n * M, torch.float64)
    nd.nd_ldos_moments(g, None, k, M, seed, 0, ld)
    C_dev = ld.view(g.n, M)[torch.from_numpy(nodes).cuda()].contiguous()
    del ld
    torch.cuda.empty_cache()
    C = C_dev.cpu().numpy()
    assert np.all(C[:, 0] == 1.0)
    e = np.abs(C - G["ldos"])
    i, m = np.unravel_index(e.argmax(), e.shape)
    assert e.max() < 1e-5, ("per-node", float(e.max()), int(nodes[i]), int(G["node_degree"][i]), int(m))
    pd = _z(nodes.size * 50, torch.float64)
    nd.nd_reconstruct(C_dev, nodes.size, M, nd.ND_KERNEL_JACKSON, (), 50, -1.0, 1.0, pd)
    l1 = np.abs(pd.cpu().numpy().reshape(nodes.size, 50) - rc.histogram(G["ldos"], 50)).sum(axis=1)
    assert l1.max() < 1e-3, ("per-node 50-bin PDOS L1", float(l1.max()), int(nodes[l1.argmax()]))


@pytest.fixture(scope="module")
def rmat22(nd):
    import torch
    W = WORKLOADS["rmat22"]
    n, s, d = W.graph(1)
    g = nd.nd_build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    return W, g


@pytest.mark.parametrize("state", ["fp32", "fp64"])
def test_rmat22_precision_study_vs_oracle_goldens(nd, rmat22, state):
    """The precision-study workload against the fp64 oracle: all 1000
    per-probe global moments, the per-node moments of 128 stored nodes and
    the 200-bin Jackson density (Sec. 3.1, Sec. 4.1).  fp64 state within
    1e-9; fp32 state within 1e-5 up to m = 200 and the linear envelope
    beyond; density L1 within 1e-3 (the stated bar)."""
    import torch
    W, g = rmat22
    G = _golden("rmat22_oracle.npz")
    k, M, seed = W.probes, W.moments, int(G["probe_seed"])
    assert g.n == int(G["n"]) and g.nnz == int(G["nnz"])
    flags = nd.ND_STATE_FP64 if state == "fp64" else 0
    mu = _z(M, torch.float64)
    pp = _z(k * M, torch.float64)
    nd.nd_cheb_moments(g, None, k, M, seed, flags, mu, pp)
    err_pp = np.abs(pp.cpu().numpy().reshape(k, M) - G["mu_pp"])
    hist = _z(W.bins, torch.float64)
    nd.nd_reconstruct(mu, 1, M, nd.ND_KERNEL_JACKSON, (), W.bins, -1.0, 1.0, hist)
    l1 = float(np.abs(hist.cpu().numpy() - G["hist200"]).sum())
    ld = _z(g.n * M, torch.float64)
    nd.nd_ldos_moments(g, None, k, M, seed, flags, ld)
    C = ld.view(g.n, M)[torch.from_numpy(G["nodes"]).cuda()].cpu().numpy()
    del ld
    err_C = np.abs(C - G["ldos"])
    if state == "fp64":
        assert err_pp.max() < 1e-9 and err_C.max() < 1e-9, (float(err_pp.max()), float(err_C.max()))
        assert l1 < 1e-9
    else:
        _check_envelope(err_pp, M, "R-MAT-22 per-probe moments")
        _check_envelope(err_C, M, "R-MAT-22 per-node moments")
        assert l1 < 1e-3
