"""Pins for the oracle's Chebyshev moments: textbook spectra, closed forms,
exact enumeration of all Rademacher probes (CPU only)."""
import itertools

import numpy as np
import pytest

import synthgraph as sg
from oracle import graph as og
from oracle import kpm
from oracle import rng as orng


def H_of(gen):
    n, s, d = gen
    g = og.build_csr(n, s, d)
    return g, og.normalized_adjacency(g)


def test_cycle_moments():
    # C_n is 2-regular: H = A/2, eigenvalues cos(2 pi k / n) -> d_m = [n | m]
    for n in (7, 8):
        g, H = H_of(sg.cycle(n))
        M = 30
        mu, ldos = kpm.exact_moments_recurrence(H, M)
        want = np.array([1.0 if m % n == 0 else 0.0 for m in range(M)])
        assert np.allclose(mu, want, atol=1e-12)
        assert np.allclose(ldos, want[None, :], atol=1e-12)  # vertex-transitive


def test_path_complete_star_spectra():
    M = 25
    n = 9
    _, H = H_of(sg.path(n))
    lam = np.cos(np.pi * np.arange(n) / (n - 1))
    assert np.allclose(kpm.exact_moments_recurrence(H, M)[0], kpm.cheb_of_eigs(lam, M).mean(1), atol=1e-12)
    _, H = H_of(sg.complete(6))
    lam = np.array([1.0] + [-1.0 / 5] * 5)
    assert np.allclose(kpm.exact_moments_recurrence(H, M)[0], kpm.cheb_of_eigs(lam, M).mean(1), atol=1e-12)
    s = 5
    _, H = H_of(sg.star(s))
    want = np.array([(1 + (-1) ** m + (s - 1) * np.cos(m * np.pi / 2)) / (s + 1) for m in range(M)])
    assert np.allclose(kpm.exact_moments_recurrence(H, M)[0], want, atol=1e-12)


@pytest.mark.parametrize("gen", [sg.complete_bipartite(3, 5), sg.path(10), sg.cycle(12), sg.star(7)])
def test_bipartite_odd_moments_vanish(gen):
    _, H = H_of(gen)
    mu, ldos = kpm.exact_moments_recurrence(H, 21)
    assert np.allclose(mu[1::2], 0.0, atol=1e-13)
    assert np.allclose(ldos[:, 1::2], 0.0, atol=1e-13)


def test_low_moment_closed_forms():
    g, H = H_of(sg.erdos_renyi(400, 0.02, seed=7))
    mu, ldos = kpm.exact_moments_recurrence(H, 3)
    assert mu[0] == 1.0 and np.all(ldos[:, 0] == 1.0)
    assert abs(mu[1]) < 1e-15 and np.all(np.abs(ldos[:, 1]) < 1e-15)
    # Chebyshev d_2 = (2/N) sum_ij A_ij/(d_i d_j) - 1 = 2 tr(H^2)/N - 1
    assert np.isclose(mu[2], 2.0 * kpm.power_moment_2(g) - 1.0, atol=1e-13)
    assert np.allclose(ldos[:, 2], kpm.cheb_moment_2_diag(g), atol=1e-13)
    # and the power moment itself: tr(H^2)/N by dense algebra
    Hd = H.toarray()
    assert np.isclose(kpm.power_moment_2(g), np.trace(Hd @ Hd) / g.n, atol=1e-13)


@pytest.mark.parametrize("gen", [sg.erdos_renyi(300, 0.02, seed=1), sg.barabasi_albert(250, 2, seed=3, twin_pairs=10),
                                 sg.rmat(9, 8, seed=2)])
def test_eigh_equals_recurrence(gen):
    _, H = H_of(gen)
    M = 60
    mu_e, l_e = kpm.exact_moments_eig(H, M)
    mu_r, l_r = kpm.exact_moments_recurrence(H, M)
    assert np.max(np.abs(mu_e - mu_r)) < 1e-10
    assert np.max(np.abs(l_e - l_r)) < 1e-10


def test_identity_probes_give_exact_moments():
    _, H = H_of(sg.erdos_renyi(120, 0.05, seed=9))
    M = 20
    mu_r, l_r = kpm.exact_moments_recurrence(H, M)
    mu, mu_pp, C = kpm.stochastic_moments(H, np.eye(H.shape[0]), M)
    # with Z = I, (1/k) sum_j z_ij y_ij = T_m(H)_ii / N * ... : C = diag / N * N/k
    assert np.allclose(C * H.shape[0], l_r, atol=1e-12)
    assert np.allclose(mu * H.shape[0], mu_r, atol=1e-12)


def all_sign_vectors(n):
    return np.array(list(itertools.product([-1.0, 1.0], repeat=n))).T  # [n][2^n]


def test_rademacher_enumeration_is_exact():
    # averaging over every +/-1 vector makes the Hutchinson / Bekas estimators
    # exact: E[z z^T] = I over the full set
    _, H = H_of(sg.erdos_renyi(9, 0.5, seed=4))
    n = H.shape[0]
    Z = all_sign_vectors(n)
    M = 12
    mu, mu_pp, C = kpm.stochastic_moments(H, Z, M)
    mu_x, l_x = kpm.exact_moments_eig(H, M)
    assert np.allclose(mu, mu_x, atol=1e-12)
    assert np.allclose(C, l_x, atol=1e-12)
    assert np.allclose(mu_pp.mean(axis=0), mu_x, atol=1e-12)


def test_rademacher_mu0_is_one():
    g, H = H_of(sg.erdos_renyi(500, 0.01, seed=3))
    Z = orng.rademacher(g.n, 6, seed=1)
    mu, mu_pp, C = kpm.stochastic_moments(H, Z, 4)
    assert np.all(mu_pp[:, 0] == 1.0) and np.all(C[:, 0] == 1.0)


def test_variance_formulas_rademacher_exact():
    # per-probe variance of z_i (T_m z)_i over all sign vectors = closed form
    _, H = H_of(sg.erdos_renyi(8, 0.6, seed=12))
    n = H.shape[0]
    M = 6
    mu_x, l_x = kpm.exact_moments_eig(H, 2 * M)
    V = kpm.ldos_probe_variance(l_x, M, "rademacher")
    Z = all_sign_vectors(n)
    for m, Y in enumerate(kpm.cheb_vectors(H, Z, M)):
        est = Z * Y
        assert np.allclose(est.var(axis=1), V[:, m], atol=1e-12)
    # a diagonal CV cannot change a Rademacher estimate at all: g (1 - z^2) = 0
    G = np.random.default_rng(0).normal(size=(n, M))
    _, C, _ = kpm.cv_ldos(H, Z, M, G)
    assert np.allclose(C, l_x[:, :M], atol=1e-12)


def test_variance_formulas_gaussian_montecarlo():
    _, H = H_of(sg.erdos_renyi(12, 0.4, seed=5))
    n = H.shape[0]
    M = 5
    mu_x, l_x = kpm.exact_moments_eig(H, 2 * M)
    Z = orng.gaussian(n, 40000, seed=3)
    G = l_x[:, :M] + 0.1  # an imperfect control variate
    Vp = kpm.ldos_probe_variance(l_x, M, "gaussian")
    Vc = kpm.ldos_probe_variance(l_x, M, "gaussian", G)
    zz = Z * Z
    for m, Y in enumerate(kpm.cheb_vectors(H, Z, M)):
        plain = (Z * Y).var(axis=1)
        cv = (G[:, m:m + 1] * (1 - zz) + Z * Y).var(axis=1)
        assert np.allclose(plain, Vp[:, m], rtol=0.06, atol=2e-3)
        assert np.allclose(cv, Vc[:, m], rtol=0.06, atol=2e-3)
    # the perfect control variate g = diag T_m reaches the Rademacher variance
    Vr = kpm.ldos_probe_variance(l_x, M, "rademacher")
    assert np.allclose(kpm.ldos_probe_variance(l_x, M, "gaussian", l_x[:, :M]), Vr)


def test_hutchinson_error_decays():
    # sanity of the stochastic path on a mid-size graph: error ~ 1/sqrt(k)
    g, H = H_of(sg.erdos_renyi(800, 0.01, seed=8))
    M = 10
    mu_x, _ = kpm.exact_moments_eig(H, M)
    errs = []
    for k in (4, 64):
        Z = orng.rademacher(g.n, k, seed=100 + k)
        mu, _, _ = kpm.stochastic_moments(H, Z, M, ldos=False)
        errs.append(np.abs(mu - mu_x)[1:].max())
    assert errs[1] < errs[0]
    assert errs[1] < 5.0 * np.sqrt(2.0 / g.n / 64)


def test_doubling_identities():
    """T_s T_{s-1} = (T_{2s-1} + T_1)/2 and T_s^2 = (T_{2s} + T_0)/2 (product
    formula of Chebyshev polynomials, used by the KPM review the paper cites
    to halve the products for traces): per probe, the direct moments equal
    the ones formed from inner products of the vectors y_s = T_s(H) z."""
    n, s, d = sg.rmat(8, 6, seed=3)
    g = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g)
    Z = orng.rademacher(g.n, 3, 2)
    M = 41
    _, mupp, _ = kpm.stochastic_moments(H, Z, M, ldos=False)
    Y = list(kpm.cheb_vectors(H, Z, M // 2 + 1))
    dot = lambda a, b: (a * b).sum(axis=0) / g.n   # noqa: E731
    for sidx in range(1, M // 2 + 1):
        even = 2.0 * dot(Y[sidx], Y[sidx]) - dot(Y[0], Y[0])
        odd = 2.0 * dot(Y[sidx], Y[sidx - 1]) - dot(Y[1], Y[0])
        if 2 * sidx < M:
            assert np.allclose(even, mupp[:, 2 * sidx], atol=1e-12)
        assert np.allclose(odd, mupp[:, 2 * sidx - 1], atol=1e-12)


# ------------------------------------------------------------ GQL (Sec. 3.2)
from oracle import gql  # noqa: E402


def test_gql_moments_equal_kpm_up_to_degree_2k_minus_1():
    """The K-node Gauss rule integrates polynomials of degree <= 2K-1 exactly,
    so its Chebyshev moments are the KPM estimates of the same probes."""
    n, s, d = sg.rmat(9, 6, seed=2)
    g = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g)
    Z = orng.rademacher(g.n, 4, 5)
    for K in (5, 12, 30):
        rules = gql.gql_probes(H, Z, K)
        mu_g = gql.gql_moments(rules, 2 * K)
        mu_k, _, _ = kpm.stochastic_moments(H, Z, 2 * K, ldos=False)
        assert np.allclose(mu_g, mu_k, atol=1e-9)
        # degree 2K is not integrated exactly in general
    rules = gql.gql_probes(H, Z, 5)
    mu_g = gql.gql_moments(rules, 12)
    mu_k, _, _ = kpm.stochastic_moments(H, Z, 12, ldos=False)
    assert np.abs(mu_g[10:] - mu_k[10:]).max() > 1e-6


def test_gql_with_unit_probes_gives_the_pdos():
    """z = e_k (Sec. 3.2): the rule estimates the PDOS of node k, and its
    Chebyshev moments are the exact PDOS moments d_mk for m <= 2K - 1."""
    n, s, d = sg.erdos_renyi(60, 0.1, seed=4)
    g = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g)
    _, l_x = kpm.exact_moments_eig(H, 16)
    K = 8
    for k in (0, 7, g.n - 1):
        e = np.zeros((g.n, 1))
        e[k, 0] = 1.0
        rules = gql.gql_probes(H, e, K)
        tau, w = rules[0]
        assert abs(w.sum() * g.n - 1.0) < 1e-12          # weights carry |z|^2 / N
        mu = gql.gql_moments(rules, 2 * K) * g.n
        assert np.allclose(mu, l_x[k, :2 * K], atol=1e-10)


def test_gql_breakdown_and_histogram():
    # the 4-cycle has 3 distinct eigenvalues: Lanczos from a generic probe stops after 3 steps
    g = og.build_csr(*sg.cycle(4))
    H = og.normalized_adjacency(g)
    a, b = gql.lanczos(H, np.array([1.0, 1.0, -1.0, 1.0]), 10)
    assert a.size <= 3
    tau, w = gql.quadrature(a, b)
    assert set(np.round(tau, 12)) <= {-1.0, 0.0, 1.0}
    rules = gql.gql_probes(H, orng.rademacher(4, 3, 1), 10)
    h = gql.gql_histogram(rules, 4)
    assert abs(h.sum() - 1.0) < 1e-12


def test_probe_estimate_is_the_eigenweight_measure():
    """Sec. 4, error analysis: a probe z turns the spectral measure into
    sum_i w_i^2 delta(lambda - lambda_i) with w = Q^T z, so the oracle's
    per-probe moments must be that measure's Chebyshev moments (per sample,
    not only in expectation), each moment's error is at most
    (1/N) sum_i |1 - w_i^2|, and the per-node estimate is the same sum with
    the node's eigenvector entries.  T_m(lambda_i) comes from numpy's
    Chebyshev Vandermonde matrix, not from the oracle."""
    g, H = H_of(sg.barabasi_albert(300, 3, seed=5))
    lam, Q = np.linalg.eigh(H.toarray())
    M, k = 40, 8
    V = np.polynomial.chebyshev.chebvander(lam, M - 1)          # [N][M], T_m(lambda_i)
    exact = V.mean(axis=0)
    for kind in ("rademacher", "gaussian"):
        Z = orng.probes(g.n, k, 21, kind)
        _, pp, C = kpm.stochastic_moments(H, Z, M)
        W = Q.T @ Z                                               # [N][k] eigen-weights
        assert np.allclose(pp, (W * W).T @ V / g.n, rtol=0, atol=1e-11)
        Y = np.einsum("ai,im,ij->maj", Q, V, W)                   # T_m(H) z_j from the eigenbasis
        assert np.allclose(C, (Z[None] * Y).mean(axis=2).T, rtol=0, atol=1e-11)
        bound = np.abs(1.0 - W * W).sum(axis=0) / g.n             # per probe
        assert np.all(np.abs(pp - exact[None]) <= bound[:, None] + 1e-12)


def test_probe_weight_error_follows_chi_square():
    """Sec. 4, error analysis: with N_z standard-normal probes, N_z times the
    mean squared weight on an eigenvector is chi^2(N_z), so E|1 - w^2| decays
    like N_z^(-1/2).  Checked on the oracle's Gaussian probes (400 seeds, the
    top eigenvector sqrt(d)/|sqrt(d)| of a graph) against the exact
    chi-square expectation.  That expectation tends to 2 / sqrt(pi N_z): the
    mean absolute deviation of a normal of variance 2 / N_z.  The paper
    prints sqrt(2 / (pi N_z)), the same rate with a constant sqrt(2) smaller."""
    from scipy import integrate, stats

    g, _ = H_of(sg.erdos_renyi(200, 0.05, seed=3))
    q = np.sqrt(g.deg.astype(np.float64))
    q /= np.linalg.norm(q)

    def expected(nz):
        f = lambda x: abs(1.0 - x / nz) * stats.chi2.pdf(x, nz)  # noqa: E731
        return integrate.quad(f, 0.0, nz)[0] + integrate.quad(f, nz, np.inf)[0]

    for nz in (4, 32):
        vals = np.array([abs(1.0 - np.mean((q @ orng.gaussian(g.n, nz, s)) ** 2)) for s in range(400)])
        se = vals.std() / np.sqrt(vals.size)
        assert abs(vals.mean() - expected(nz)) < 4.0 * se, (nz, vals.mean(), expected(nz))
    for nz in (64, 256, 1024):
        assert abs(expected(nz) / (2.0 / np.sqrt(np.pi * nz)) - 1.0) < 1.0 / nz
