"""CPU oracle for the network density-of-states (DOS/LDOS) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under ``oracle/``: only the test suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the GPU
library (no kernels, headers, helpers or tables); both sides consume the same
seeded edge lists from :mod:`synthgraph`, and each implements the counter-based
probe generator (SplitMix64) on its own from its published definition.

Everything here is plain, slow and fp64 (unless the method fixes a precision),
written from the paper, Dong, Benson & Bindel, "Network Density of States",
KDD 2019 (arXiv:1905.09758):

* :mod:`oracle.graph`        -- simple symmetric graph, CSR, normalized adjacency (Sec. 2.1)
* :mod:`oracle.rng`          -- probe vectors (Sec. 3.1, probe estimators)
* :mod:`oracle.kpm`          -- Chebyshev moments, exact and stochastic (Sec. 3.1)
* :mod:`oracle.twins`        -- twin motifs and probe projection (Sec. 3.4)
* :mod:`oracle.gql`          -- Gauss quadrature and Lanczos, GQL (Sec. 3.2)
* :mod:`oracle.reconstruct`  -- Jackson damping, density, histogram (Sec. 2.2, 3.1, 4.1)
* :mod:`oracle.cv`           -- learned control variate: features, MLP, estimator
                                (not in the paper; parity unpinned by the paper)
"""
