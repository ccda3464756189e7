"""The allocation-free entry point (nd_cheb_moments_noalloc) against the
allocating one, through the C ABI (needs an MI355X).

Two calls in a row on the fixed workspace, the second with a smaller input
(fewer nodes, probes and moments), each compared with nd_cheb_moments on the
same inputs (same kernels: identical bits) and with the oracle (fp32 bar of
the global moments); plus the host-side refusals (workspace need above the
limit, no schedule yet, ND_TIME_STEPS)."""
import numpy as np
import pytest

import synthgraph as sg
from oracle import graph as og
from oracle import kpm, rng as orng

pytestmark = pytest.mark.gpu

TOL_MU = 1e-5


def _zeros(n, dtype):
    import torch
    return torch.zeros(n, dtype=dtype, device="cuda")


def _pair(nd, n, s, d, k, M, seed, flags):
    """(allocating mu, mu_pp), (allocation-free mu, mu_pp) and the oracle's mu_pp."""
    import torch
    g = nd.nd_build_csr(n, s, d)
    mu_a, pp_a = _zeros(M, torch.float64), _zeros(k * M, torch.float64)
    nd.nd_cheb_moments(g, None, k, M, seed, flags, mu_a, pp_a)
    # the fixed workspace keeps the previous call's contents: fill the outputs
    # with garbage so that a missed write shows
    mu_b = torch.full((M,), 7.0, dtype=torch.float64, device="cuda")
    pp_b = torch.full((k * M,), -3.0, dtype=torch.float64, device="cuda")
    nd.nd_cheb_moments_noalloc(g, k, M, seed, flags, mu_b, pp_b)
    mu_c = torch.full((M,), 5.0, dtype=torch.float64, device="cuda")
    nd.nd_cheb_moments_noalloc(g, k, M, seed, flags, mu_c)          # per-probe sums in the workspace
    torch.cuda.synchronize()
    g_or = og.build_csr(n, s, d)
    Z = orng.rademacher(g_or.n, k, seed) if not (flags & nd.ND_PROBE_GAUSSIAN) else orng.gaussian(g_or.n, k, seed)
    mu_o, pp_o, _ = kpm.stochastic_moments(og.normalized_adjacency(g_or), Z, M, ldos=False)
    return g, (mu_a.cpu().numpy(), pp_a.cpu().numpy()), (mu_b.cpu().numpy(), pp_b.cpu().numpy()), \
        mu_c.cpu().numpy(), (mu_o, pp_o)


@pytest.mark.parametrize("flags_name", ["rademacher", "fp64", "doubling", "gaussian"])
def test_noalloc_two_calls_second_smaller(nd, flags_name):
    flags = {"rademacher": 0, "fp64": nd.ND_STATE_FP64, "doubling": nd.ND_MOMENT_DOUBLING,
             "gaussian": nd.ND_PROBE_GAUSSIAN}[flags_name]
    cases = [(sg.rmat(14, 8, seed=2), 40, 120, 3), (sg.erdos_renyi(2000, 0.005, seed=1), 20, 100, 5)]
    for (n, s, d), k, M, seed in cases:
        g, (mu_a, pp_a), (mu_b, pp_b), mu_c, (mu_o, pp_o) = _pair(nd, n, s, d, k, M, seed, flags)
        assert np.array_equal(mu_a, mu_b) and np.array_equal(pp_a, pp_b)
        assert np.array_equal(mu_a, mu_c)
        tol = TOL_MU * (10 if flags_name == "gaussian" else 1)
        assert np.max(np.abs(mu_b - mu_o)) < tol
        assert np.max(np.abs(pp_b.reshape(k, M) - pp_o)) < tol


def test_noalloc_refusals(nd):
    import torch
    # a graph whose recurrence state alone exceeds the fixed workspace
    n, s, d = sg.barabasi_albert(400_000, 3, seed=1)
    g = nd.nd_build_csr(n, s, d)
    M = 4
    mu = _zeros(M, torch.float64)
    with pytest.raises(nd.NDError) as e:                  # no schedule for 16 probes yet
        nd.nd_cheb_moments_noalloc(g, 16, M, 1, 0, mu)
    assert e.value.status == nd.ND_EINVAL and "schedule" in str(e.value)
    nd.nd_cheb_moments(g, None, 16, M, 1, 0, mu)
    with pytest.raises(nd.NDError) as e:                  # 3 x 400k x 16 x 4 bytes > 64 MiB
        nd.nd_cheb_moments_noalloc(g, 16, M, 1, 0, mu)
    assert e.value.status == nd.ND_EINVAL and "bytes of workspace" in str(e.value)
    n, s, d = sg.erdos_renyi(2000, 0.005, seed=1)
    g = nd.nd_build_csr(n, s, d)
    nd.nd_cheb_moments(g, None, 8, M, 1, 0, mu)
    with pytest.raises(nd.NDError) as e:
        nd.nd_cheb_moments_noalloc(g, 8, M, 1, nd.ND_TIME_STEPS, mu)
    assert e.value.status == nd.ND_EINVAL
    nd.nd_cheb_moments_noalloc(g, 8, M, 1, 0, mu)         # still usable after the refusals
    assert mu.cpu().numpy()[0] == pytest.approx(1.0, abs=1e-12)
