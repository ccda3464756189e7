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
