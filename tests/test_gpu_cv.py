"""Learned control variate on the GPU vs the fp64 oracle (needs an MI355X).

The control variate is not in the paper: features, MLP and Adam are pinned to
their definitions (parity unpinned by the paper); the estimator's variance is
pinned to the closed form of the oracle."""
import numpy as np
import pytest

import synthgraph as sg
from synthgraph.mlp_init import init_params
from synthgraph import workloads
from oracle import graph as og
from oracle import cv as ocv
from oracle import kpm

pytestmark = pytest.mark.gpu


def _t(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


GRAPHS = {
    "er": lambda: sg.erdos_renyi(600, 0.02, seed=3),
    "ba_twins": lambda: sg.barabasi_albert(900, 3, seed=2, twin_pairs=40),
    "rmat": lambda: sg.rmat(10, 8, seed=5),
    "star": lambda: sg.star(700),
    "sbm": lambda: sg.sbm(1200, 0.05, 0.005, seed=1),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_features(nd, name):
    import torch
    n, s, d = GRAPHS[name]()
    g = nd.nd_build_csr(n, s, d)
    want = ocv.log_scale(ocv.raw_features(og.build_csr(n, s, d)))
    f = torch.empty(g.n * 5, dtype=torch.float32, device="cuda")
    nd.nd_node_features(g, f)
    got = f.cpu().numpy().reshape(g.n, 5)
    assert np.allclose(got, want, rtol=1e-6, atol=1e-6)
    mean = want.mean(axis=0).astype(np.float32)
    std = (want.std(axis=0) + 0.5).astype(np.float32)
    nd.nd_node_features(g, f, _t(mean, torch.float32), _t(std, torch.float32))
    got2 = f.cpu().numpy().reshape(g.n, 5)
    assert np.allclose(got2, (want - mean) / std, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_cv_exact_diag(nd, name):
    """T_0..T_3(H)_ii from closed forms on the device against the oracle's
    exact diagonal (the recurrence with Z = I, Sec. 3.1)."""
    import torch
    n, s, d = GRAPHS[name]()
    g = nd.nd_build_csr(n, s, d)
    g_or = og.build_csr(n, s, d)
    _, want = kpm.exact_moments_recurrence(og.normalized_adjacency(g_or), 4)
    ld = 7
    out = torch.full((g.n * ld,), 3.0, dtype=torch.float32, device="cuda")
    nd.nd_cv_exact_diag(g, out, ld, 4)
    got = out.cpu().numpy().reshape(g.n, ld)
    assert np.max(np.abs(got[:, :4] - want)) < 1e-6
    assert np.all(got[:, 4:] == 3.0)                      # other columns untouched
    assert np.all(got[:, 0] == 1.0) and np.all(got[:, 1] == 0.0)


def test_features_beyond_lds_bitmaps(nd):
    """A graph of more than 524288 nodes: the neighbourhood bitmaps move to a
    device workspace; features against the oracle."""
    import torch
    n, s, d = sg.erdos_renyi(600_000, 5.0 / 600_000, seed=4)
    g = nd.nd_build_csr(n, s, d)
    assert g.n > 524288
    g_or = og.build_csr(n, s, d)
    want = ocv.log_scale(ocv.raw_features(g_or))
    f = torch.empty(g.n * 5, dtype=torch.float32, device="cuda")
    nd.nd_node_features(g, f)
    assert np.allclose(f.cpu().numpy().reshape(g.n, 5), want, rtol=1e-6, atol=1e-6)
    out = torch.zeros(g.n * 4, dtype=torch.float32, device="cuda")
    nd.nd_cv_exact_diag(g, out, 4, 4)
    t2 = kpm.cheb_moment_2_diag(g_or)
    assert np.max(np.abs(out.cpu().numpy().reshape(g.n, 4)[:, 2] - t2)) < 1e-6


def test_motif_diag(nd):
    """The exact motif part of the diagonal for every kind of class, against
    the oracle's classes, eigenvalues and Chebyshev values (Sec. 3.4)."""
    import torch
    from oracle import twins
    n, s, d = sg.barabasi_albert(2000, 1, seed=4)             # a tree: open and pendant twins
    n, s, d = sg.plant_adjacent_pairs(n, s, d, 30, seed=9)     # closed twins
    g = nd.nd_build_csr(n, s, d)
    g_or = og.build_csr(n, s, d)
    kinds = nd.ND_TWINS_OPEN | nd.ND_TWINS_CLOSED | nd.ND_PENDANTS | nd.ND_HUBPATHS
    m = nd.nd_motif_filter(g, 3, kinds)
    cls, lam = twins.motif_classes(g_or, {"open", "closed", "pendants", "hubpaths"})
    M, ld = 12, 15
    want = np.full((g_or.n, ld), 0.25)
    for c, sig in zip(cls, lam):
        t = sum(f * twins.cheb_at(x, M) for x, f in twins.signature(sig))
        want[np.asarray(c), :M] += -2.0 * (1.0 - 1.0 / len(c)) * t
    out = torch.full((g.n * ld,), 0.25, dtype=torch.float32, device="cuda")
    nd.nd_motif_diag(m, out, ld, M, -2.0)
    assert np.max(np.abs(out.cpu().numpy().reshape(g.n, ld) - want)) < 1e-6


def test_control_variate_with_twin_classes_is_refused(nd):
    """A projected probe entry of a class member has mean square 1/|C|, not 1,
    so g (1 - z~_i^2) would bias that row: cv_g together with motifs that
    hold classes is refused; motifs without classes are accepted."""
    import torch
    n, s, d = GRAPHS["ba_twins"]()
    g = nd.nd_build_csr(n, s, d)
    m = nd.nd_motif_filter(g, 1)
    assert m.n_classes > 0
    M, k = 8, 4
    cvg = torch.zeros(g.n * M, dtype=torch.float32, device="cuda")
    ld = torch.zeros(g.n * M, dtype=torch.float64, device="cuda")
    with pytest.raises(nd.NDError) as e:
        nd.nd_ldos_moments(g, m, k, M, 3, nd.ND_PROBE_GAUSSIAN, ld, cv_g=cvg)
    assert e.value.status == nd.ND_EINVAL
    n2, s2, d2 = sg.cycle(50)                       # no twins: an empty class list
    g2 = nd.nd_build_csr(n2, s2, d2)
    m2 = nd.nd_motif_filter(g2, 1)
    assert m2.n_classes == 0
    cv2 = torch.zeros(g2.n * M, dtype=torch.float32, device="cuda")
    ld2 = torch.zeros(g2.n * M, dtype=torch.float64, device="cuda")
    nd.nd_ldos_moments(g2, m2, k, M, 3, nd.ND_PROBE_GAUSSIAN, ld2, cv_g=cv2)


def test_ldos_variance(nd):
    """The library's variance reduction against the per-probe sample variance
    computed from the oracle's estimates on the same probes."""
    import torch
    from oracle import rng as orng
    n, s, d = GRAPHS["rmat"]()
    g = nd.nd_build_csr(n, s, d)
    g_or = og.build_csr(n, s, d)
    k, M = 24, 20
    G = np.random.default_rng(2).normal(size=(g_or.n, M)).astype(np.float32)
    Z = orng.gaussian(g_or.n, k, 9)
    _, C, S2 = kpm.cv_ldos(og.normalized_adjacency(g_or), Z, M, G.astype(np.float64))
    s2 = k / (k - 1.0) * (S2 - C * C)
    ld = _t(C, torch.float64)
    sq = _t(S2, torch.float64)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    per_m = torch.empty(M, dtype=torch.float64, device="cuda")
    nd.nd_ldos_variance(ld, sq, g_or.n, M, 1, k, out, per_m)
    assert abs(out.item() - s2[:, 1:].mean()) < 1e-12 * (1 + abs(s2[:, 1:].mean()))
    assert np.allclose(per_m.cpu().numpy(), s2.mean(axis=0), rtol=1e-12, atol=1e-14)


def test_column_stats(nd):
    import torch
    x = np.random.default_rng(0).normal(3.0, 2.0, size=(100_003, 5)).astype(np.float32)
    mean = torch.empty(5, dtype=torch.float32, device="cuda")
    std = torch.empty(5, dtype=torch.float32, device="cuda")
    nd.nd_column_stats(_t(x, torch.float32), x.shape[0], 5, mean, std)
    x64 = x.astype(np.float64)
    assert np.allclose(mean.cpu().numpy(), x64.mean(axis=0), rtol=1e-6)
    assert np.allclose(std.cpu().numpy(), x64.std(axis=0), rtol=1e-5)


@pytest.mark.parametrize("n,n_out", [(1, 64), (97, 64), (1000, 7), (333, 128)])
def test_mlp_forward(nd, n, n_out):
    import torch
    p = init_params(11, n_out)
    x = np.random.default_rng(n).normal(size=(n, 5)).astype(np.float32)
    out = torch.empty(n * n_out, dtype=torch.float32, device="cuda")
    nd.nd_mlp_forward(_t(p, torch.float32), _t(x, torch.float32), n, n_out, out)
    want = ocv.forward(p.astype(np.float64), x.astype(np.float64), n_out)
    got = out.cpu().numpy().reshape(n, n_out)
    assert np.max(np.abs(got - want)) <= 1e-4 * (1.0 + np.max(np.abs(want)))


@pytest.mark.parametrize("n,n_out,use_idx", [(64, 64, False), (4096, 64, True), (77, 13, True)])
def test_mlp_grad(nd, n, n_out, use_idx):
    import torch
    rng = np.random.default_rng(n + n_out)
    p = init_params(5, n_out).astype(np.float32)
    p[-n_out:] = rng.normal(size=n_out).astype(np.float32) * 0.1
    rows = 2 * n + 5
    x = rng.normal(size=(rows, 5)).astype(np.float32)
    y = rng.normal(size=(rows, n_out + 3)).astype(np.float32)  # ld_target > n_out
    idx = rng.integers(0, rows, size=n).astype(np.int32) if use_idx else np.arange(n, dtype=np.int32)
    grad = torch.empty(nd.n_params(n_out), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    nd.nd_mlp_grad(_t(p, torch.float32), _t(x, torch.float32), _t(y, torch.float32), n_out + 3,
                   _t(idx, torch.int32) if use_idx else None, n, n_out, grad, loss)
    l_o, g_o = ocv.mse_grad(p.astype(np.float64), x[idx].astype(np.float64),
                            y[idx, :n_out].astype(np.float64), n_out)
    g = grad.cpu().numpy()
    assert abs(loss.item() - l_o) <= 1e-5 * abs(l_o)
    assert np.max(np.abs(g - g_o)) <= 1e-3 * np.max(np.abs(g_o)) + 1e-6


def test_adam(nd):
    import torch
    rng = np.random.default_rng(1)
    P = 1000
    p, m, v, g = (rng.normal(size=P).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    dp, dm, dv = _t(p, torch.float32), _t(m, torch.float32), _t(v, torch.float32)
    for t in (1, 2, 3):
        nd.nd_adam_step(dp, dm, dv, _t(g, torch.float32), P, t, 1e-3)
        p, m, v = ocv.adam_step(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64), g, t, 1e-3)
    assert np.allclose(dp.cpu().numpy(), p, rtol=1e-5, atol=1e-6)
    assert np.allclose(dv.cpu().numpy(), v, rtol=1e-5, atol=1e-9)


def test_cv_variance_matches_closed_form(nd):
    """Per-probe variance of the Gaussian estimator with a fixed control
    variate g equals V_R + 2 (b - g)^2 (oracle, from exact PDOS moments)."""
    import torch
    n, s, d = sg.erdos_renyi(400, 0.03, seed=9)
    g_or = og.build_csr(n, s, d)
    M = 8
    _, l_x = kpm.exact_moments_eig(og.normalized_adjacency(g_or), 2 * M)
    G = (l_x[:, :M] + 0.2 * np.random.default_rng(0).normal(size=(g_or.n, M))).astype(np.float32)
    g = nd.nd_build_csr(n, s, d)
    k = 4000
    ld = torch.empty(g.n * M, dtype=torch.float64, device="cuda")
    sq = torch.empty(g.n * M, dtype=torch.float64, device="cuda")
    nd.nd_ldos_moments(g, None, k, M, 3, nd.ND_PROBE_GAUSSIAN, ld, cv_g=_t(G, torch.float32), ldos_sq=sq)
    s2 = ((sq - ld * ld) * (k / (k - 1.0))).cpu().numpy().reshape(g.n, M)
    want = kpm.ldos_probe_variance(l_x, M, "gaussian", G.astype(np.float64))
    # sample variances of 4000 probes: ~ sqrt(2/k) relative error per entry; compare averages
    assert np.allclose(s2[:, 1:].mean(axis=0), want[:, 1:].mean(axis=0), rtol=0.05, atol=1e-3)
    # unbiased: the estimate agrees with the exact PDOS moments
    C = ld.cpu().numpy().reshape(g.n, M)
    assert np.max(np.abs(C.mean(axis=0) - l_x[:, :M].mean(axis=0))) < 0.02


def test_training_reduces_gaussian_variance(nd):
    """Train on a few small graphs of the study's families, then the learned
    control variate lowers the Gaussian per-probe variance on held-out
    graphs; with +/-1 probes it changes nothing (the estimator is identical)."""
    import torch
    from paper_1905_09758_amd import cv
    M = 16
    specs = workloads.cv_graph_specs(8, seed=1, n_lo=2000, n_hi=6000)
    held = workloads.cv_graph_specs(2, seed=99, n_lo=2000, n_hi=6000)
    graphs = [nd.nd_build_csr(*workloads.cv_graph(sp)) for sp in specs]
    targets = [cv.ldos_targets(g, 256, M, seed=5 + i) for i, g in enumerate(graphs)]
    model, hist = cv.train(graphs, targets, M, init_params(0, M), steps=600, batch=2048, lr=3e-3, seed=0,
                           log_every=100)
    assert hist[-1][1] < hist[0][1]
    for sp in held:
        g = nd.nd_build_csr(*workloads.cv_graph(sp))
        gcv = cv.predict(g, model)
        v_plain = cv.probe_variance(g, M, 512, 7, gaussian=True)
        v_cv = cv.probe_variance(g, M, 512, 7, gaussian=True, cv_g=gcv)
        assert v_cv < 0.9 * v_plain, (sp, v_plain, v_cv)
        r_plain = cv.probe_variance(g, M, 128, 8, gaussian=False)
        r_cv = cv.probe_variance(g, M, 128, 8, gaussian=False, cv_g=gcv)
        assert abs(r_cv - r_plain) <= 1e-6 * r_plain
