"""Gauss quadrature and Lanczos (Sec. 3.2) on the GPU against the oracle
(needs an MI355X).  The Lanczos coefficients with fp64 vectors match the
oracle's plain fp64 Lanczos; the rules' Chebyshev moments equal the KPM
estimates of the same probes up to degree 2K-1 (fp64 and fp32 vectors); the
density helpers bin and integrate the rules exactly."""
import numpy as np
import pytest

import synthgraph as sg
from oracle import graph as og
from oracle import kpm, gql, rng as orng, twins

pytestmark = pytest.mark.gpu

GRAPHS = {
    "er2000": lambda: sg.erdos_renyi(2000, 0.005, seed=1),
    "ba_twins": lambda: sg.barabasi_albert(3000, 2, seed=5, twin_pairs=150),
    "rmat12": lambda: sg.rmat(12, 8, seed=7),
    "star": lambda: sg.star(3000),          # three distinct eigenvalues: early stop
    "ws": lambda: sg.watts_strogatz(1500, 4, 0.3, seed=2),
}


@pytest.fixture(scope="module", params=sorted(GRAPHS))
def case(request, nd):
    n, s, d = GRAPHS[request.param]()
    g_or = og.build_csr(n, s, d)
    return request.param, g_or, og.normalized_adjacency(g_or), nd.nd_build_csr(n, s, d)


def _run(nd, g, motifs, k, K, seed, flags):
    import torch
    z = lambda dt: torch.zeros(k * K, dtype=dt, device="cuda")   # noqa: E731
    nodes, weights, alpha, beta = z(torch.float64), z(torch.float64), z(torch.float64), z(torch.float64)
    steps = torch.zeros(k, dtype=torch.int32, device="cuda")
    nd.nd_gql(g, motifs, k, K, seed, flags, nodes, weights, steps, alpha, beta)
    return nodes, weights, steps, alpha, beta


def _rules(nodes, weights, steps, k, K):
    n, w, s = (x.cpu().numpy() for x in (nodes, weights, steps))
    n, w = n.reshape(k, K), w.reshape(k, K)
    return [(n[j, :s[j]], w[j, :s[j]]) for j in range(k)]


def test_lanczos_fp64_matches_oracle(case, nd):
    name, g_or, H, g = case
    k, K = 6, 12
    Z = orng.rademacher(g_or.n, k, 3)
    nodes, weights, steps, alpha, beta = _run(nd, g, None, k, K, 3, nd.ND_STATE_FP64)
    al, be, st = (x.cpu().numpy() for x in (alpha, beta, steps))
    al, be = al.reshape(k, K), be.reshape(k, K)
    for j in range(k):
        a_o, b_o = gql.lanczos(H, Z[:, j], K)
        assert st[j] == a_o.size, (name, j, st[j], a_o.size)
        assert np.max(np.abs(al[j, :a_o.size] - a_o)) < 1e-9
        assert np.max(np.abs(be[j, :b_o.size] - b_o)) < 1e-9
        assert np.all(al[j, a_o.size:] == 0.0)
    if name == "star":
        assert np.all(st <= 3)
    rules = _rules(nodes, weights, steps, k, K)
    mu_o, _, _ = kpm.stochastic_moments(H, Z, 2 * K, ldos=False)
    assert np.max(np.abs(gql.gql_moments(rules, 2 * K) - mu_o)) < 1e-9
    for (tau, w), (t_o, w_o) in zip(rules, gql.gql_probes(H, Z, K)):
        assert np.allclose(np.sort(tau), np.sort(t_o), atol=1e-9)
        assert abs(w.sum() - w_o.sum()) < 1e-12


@pytest.mark.parametrize("K", [20, 40])
def test_gql_fp32_moments_equal_kpm(case, nd, K):
    import torch
    name, g_or, H, g = case
    k = 16
    Z = orng.rademacher(g_or.n, k, 11)
    nodes, weights, steps, _, _ = _run(nd, g, None, k, K, 11, 0)
    mu = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
    hist = torch.zeros(50, dtype=torch.float64, device="cuda")
    nd.nd_gql_density(nodes, weights, k, K, 2 * K, mu, 50, -1.0, 1.0, hist)
    mu_o, _, _ = kpm.stochastic_moments(H, Z, 2 * K, ldos=False)
    assert np.max(np.abs(mu.cpu().numpy() - mu_o)) < 1e-5
    # the density helpers on the GPU's own rules: exact up to summation order
    rules = _rules(nodes, weights, steps, k, K)
    assert np.max(np.abs(mu.cpu().numpy() - gql.gql_moments(rules, 2 * K))) < 1e-12
    assert np.max(np.abs(hist.cpu().numpy() - gql.gql_histogram(rules, 50))) < 1e-12
    assert abs(hist.cpu().numpy().sum() - 1.0) < 1e-12


def test_gql_filtered_and_gaussian(nd):
    import torch
    n, s, d = sg.barabasi_albert(3000, 2, seed=5, twin_pairs=150)
    g_or = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g_or)
    g = nd.nd_build_csr(n, s, d)
    m = nd.nd_motif_filter(g, 2, 0x3)
    cls = twins.twin_classes(g_or, "both")
    k, K = 8, 15
    Z = orng.rademacher(g_or.n, k, 6)
    nodes, weights, steps, _, _ = _run(nd, g, m, k, K, 6, nd.ND_STATE_FP64)
    rules = _rules(nodes, weights, steps, k, K)
    _, mu_s, _, _ = twins.filtered_moments(H, Z, 2 * K, cls, ldos=False,
                                           lambdas=[twins.class_eigenvalue(g_or, c) for c in cls])
    assert np.max(np.abs(gql.gql_moments(rules, 2 * K) - mu_s)) < 1e-9
    # Gaussian probes from the oracle's own generator.  Its libm may differ
    # from the device's by an ulp before the fp32 rounding (a probe entry
    # then differs by <= 4e-7 relative), which moves a moment by at most
    # ~2 * 4e-7 * max|z| * rms(z) ~ 1e-5; equal entries leave it exact.
    Zg = orng.gaussian(g_or.n, k, 9)
    nodes, weights, steps, _, _ = _run(nd, g, None, k, K, 9, nd.ND_PROBE_GAUSSIAN | nd.ND_STATE_FP64)
    rules = _rules(nodes, weights, steps, k, K)
    mu_g, _, _ = kpm.stochastic_moments(H, Zg, 2 * K, ldos=False)
    assert np.max(np.abs(gql.gql_moments(rules, 2 * K) - mu_g)) < 1e-5


def test_gql_errors(nd):
    import torch
    n, s, d = sg.cycle(8)
    g = nd.nd_build_csr(n, s, d)
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(nd.NDError):
        nd.nd_gql(g, None, 2, 4, 1, nd.ND_MOMENT_DOUBLING, buf, buf)
    with pytest.raises(nd.NDError):
        nd.nd_gql(g, None, 2, 0, 1, 0, buf, buf)
    with pytest.raises(nd.NDError):
        nd.nd_gql_density(buf, buf, 2, 4)


@pytest.mark.parametrize("state", ["fp32", "fp64"])
def test_gql_pdos_unit_probes(nd, state):
    """GQL from e_v (Sec. 3.2): the rule's moments are the exact PDOS moments
    of v up to degree 2K-1; weights sum to 1."""
    import torch
    n, s, d = sg.barabasi_albert(1500, 2, seed=3, twin_pairs=20)
    g_or = og.build_csr(n, s, d)
    g = nd.nd_build_csr(n, s, d)
    K = 10
    _, l_x = kpm.exact_moments_eig(og.normalized_adjacency(g_or), 2 * K)
    rng = np.random.default_rng(4)
    sel = np.concatenate([[int(np.argmax(g_or.deg))], rng.choice(g_or.n, 69, replace=False)]).astype(np.int32)
    kk = sel.size * K
    nodes = torch.zeros(kk, dtype=torch.float64, device="cuda")
    weights = torch.zeros(kk, dtype=torch.float64, device="cuda")
    steps = torch.zeros(sel.size, dtype=torch.int32, device="cuda")
    flags = nd.ND_STATE_FP64 if state == "fp64" else 0
    nd.nd_gql_pdos(g, torch.from_numpy(sel).cuda(), K, flags, nodes, weights, steps)
    n_, w_, s_ = (x.cpu().numpy() for x in (nodes, weights, steps))
    n_, w_ = n_.reshape(sel.size, K), w_.reshape(sel.size, K)
    tol = 1e-9 if state == "fp64" else 1e-5
    for j, v in enumerate(sel):
        rule = [(n_[j, :s_[j]], w_[j, :s_[j]])]
        assert abs(w_[j].sum() - 1.0) < 1e-9
        assert np.max(np.abs(gql.gql_moments(rule, 2 * K) - l_x[v, :2 * K])) < tol
