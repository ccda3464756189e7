"""The benchmark and parity workloads: seeded synthetic inputs with the shapes
of the paper's experiments (the paper's SNAP / RODGER datasets are not
available, so these stand in for them).

Each recipe returns ``(n_nodes, src, dst)`` edge lists from
:mod:`synthgraph` plus the run parameters.
"""
from __future__ import annotations

from dataclasses import dataclass

import synthgraph as sg


@dataclass(frozen=True)
class Workload:
    name: str
    probes: int
    moments: int
    bins: int
    ldos: bool
    filter_twins: bool
    describe: str

    def graph(self, seed: int = 1):
        return GENERATORS[self.name](seed)


GENERATORS = {
    # G(2000, 0.005): the small case checked against a dense eigendecomposition
    "er2000": lambda seed: sg.erdos_renyi(2000, 0.005, seed=seed),
    # Barabasi-Albert n = 10^6, m = 5, plus 5% extra leaves in pairs on shared
    # random hubs (25,000 planted twin pairs); stands in for motif-rich graphs
    "ba1m_twins": lambda seed: sg.barabasi_albert(1_000_000, 5, seed=seed, twin_pairs=25_000),
    # R-MAT scale 27, edge factor 8, (0.57, 0.19, 0.19, 0.05): ~1e9 edges;
    # stands in for the billion-edge social networks
    "rmat27": lambda seed: sg.rmat(27, 8, seed=seed),
    # R-MAT scale 22, edge factor 16, same parameters: the precision study
    "rmat22": lambda seed: sg.rmat(22, 16, seed=seed),
    # smaller R-MAT used as the oracle's timing sample for the R-MAT workloads
    "rmat20": lambda seed: sg.rmat(20, 8, seed=seed),
}

WORKLOADS = {
    "er2000": Workload("er2000", 20, 100, 100, False, False,
                       "Erdos-Renyi G(2000, 0.005), 20 Rademacher probes, 100 moments, 100 bins"),
    "ba1m_twins": Workload("ba1m_twins", 64, 500, 100, True, True,
                           "Barabasi-Albert n=1e6 m=5 + 25k planted twin pairs, 64 Rademacher probes, "
                           "500 moments, global DOS + per-node LDOS, twin filter on"),
    "rmat27": Workload("rmat27", 16, 200, 100, False, False,
                       "R-MAT scale 27 ef 8 (0.57,0.19,0.19,0.05), 16 Rademacher probes, 200 moments, global DOS"),
    "rmat22": Workload("rmat22", 32, 1000, 200, False, False,
                       "R-MAT scale 22 ef 16, 32 Rademacher probes, 1000 moments, global DOS"),
}


# ---------------------------------------------------------------- control-variate graphs
# Families and parameters of the learned-control-variate study: Erdos-Renyi
# with mean degree U[4, 20]; Barabasi-Albert with m in {2..6}; R-MAT with
# edge factor 8 or 16 at scale ceil(log2 n), endpoints reduced mod n; a
# 4-block SBM with p_in = 0.01, p_out = 0.001.  n is uniform in [n_lo, n_hi].
CV_FAMILIES = ("er", "ba", "rmat", "sbm")


def cv_graph_specs(count: int, seed: int, n_lo: int = 10_000, n_hi: int = 200_000):
    """`count` (family, n, parameter, graph seed) tuples, families in turn."""
    import numpy as np
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        fam = CV_FAMILIES[i % len(CV_FAMILIES)]
        n = int(rng.integers(n_lo, n_hi + 1))
        if fam == "er":
            par = float(rng.uniform(4.0, 20.0))
        elif fam == "ba":
            par = int(rng.integers(2, 7))
        elif fam == "rmat":
            par = int(rng.choice([8, 16]))
        else:
            par = 0
        specs.append((fam, n, par, int(rng.integers(1, 2**31 - 1))))
    return specs


def cv_graph(spec):
    fam, n, par, gseed = spec
    if fam == "er":
        return sg.erdos_renyi(n, par / (n - 1), seed=gseed)
    if fam == "ba":
        return sg.barabasi_albert(n, par, seed=gseed)
    if fam == "rmat":
        scale = max(1, (n - 1).bit_length())
        return sg.rmat(scale, par, seed=gseed, n_mod=n)
    if fam == "sbm":
        return sg.sbm(n, 0.01, 0.001, seed=gseed)
    raise ValueError(fam)
