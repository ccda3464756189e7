"""Writes the oracle's expected values for the full-size parity tests.

Every number stored here comes from ``oracle/`` (plain fp64 numpy/scipy, and
its C leg for the billion-edge graph) run on the seeded synthetic workloads of
``synthgraph``; nothing is read from the HIP library.  Run from the repository
root on a CPU host (the R-MAT scale-27 leg needs about 40 GB of memory):

    python tests/golden/make_goldens.py ba1m rmat22 rmat27

Outputs (npz, fp64):

* ``ba1m_twins_oracle.npz`` -- BA n=10^6 m=5 + 25k planted twin pairs, 64
  Rademacher probes (seed 1), all 500 moments: per-probe global moments
  without and with the open-twin filter (smooth part) and the filtered full
  moments (Sec. 3.1 eqn doscoeff, Sec. 3.4); per-node moments (eqn pdoscoeff)
  of 192 nodes -- the 64 of largest degree, 64 twin-class members, 64 others
  -- without and with the filter.
* ``rmat22_oracle.npz`` -- R-MAT scale 22 ef 16, 32 probes (seed 1), all 1000
  moments per probe, per-node moments of 128 nodes (the 32 of largest degree
  and 96 others), and the 200-bin Jackson density of the mean moments
  (Sec. 3.1, Sec. 4.1).
* ``rmat27_oracle.npz`` -- R-MAT scale 27 ef 8, 16 probes (seed 1), all 200
  moments per probe and per-node moments of 64 nodes (the 16 of largest
  degree -- rows that the device splits across wavefronts -- and 48 others);
  about 90 minutes on 8 cores.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from synthgraph.workloads import WORKLOADS  # noqa: E402
from oracle import graph as og, kpm, rng as orng, twins, reconstruct as rc  # noqa: E402

PROBE_SEED = 1
GRAPH_SEED = 1


def _log(msg: str) -> None:
    print("[make_goldens %s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


def _pick_nodes(deg: np.ndarray, n_top: int, n_rand: int, seed: int, exclude=None) -> np.ndarray:
    """The n_top nodes of largest degree (ties by id) and n_rand others drawn
    without replacement from the rest."""
    order = np.lexsort((np.arange(deg.size), -deg))
    top = order[:n_top]
    rest = np.ones(deg.size, dtype=bool)
    rest[top] = False
    if exclude is not None:
        rest[exclude] = False
    rng = np.random.default_rng(seed)
    others = rng.choice(np.flatnonzero(rest), n_rand, replace=False)
    return np.sort(np.concatenate([top, others])).astype(np.int64)


def make_ba1m() -> None:
    W = WORKLOADS["ba1m_twins"]
    k, M = W.probes, W.moments
    n, s, d = W.graph(GRAPH_SEED)
    g = og.build_csr(n, s, d)
    del s, d
    H = og.normalized_adjacency(g)
    cls = twins.twin_classes(g)
    members = np.concatenate([np.asarray(c) for c in cls]).astype(np.int64)
    rng = np.random.default_rng(7)
    twin_pick = rng.choice(members, 64, replace=False)
    nodes = np.union1d(_pick_nodes(g.deg, 64, 64, 11, exclude=members), twin_pick).astype(np.int64)
    Z = orng.rademacher(g.n, k, PROBE_SEED)
    _log("BA-1M: n=%d nnz=%d classes=%d; plain run" % (g.n, g.nnz, len(cls)))
    t0 = time.time()
    _, pp_plain, C = kpm.stochastic_moments(H, Z, M, ldos=True)
    ld_plain = C[nodes].copy()
    del C
    _log("BA-1M plain done in %.0f s; filtered run" % (time.time() - t0))
    mu_full, _, pp_smooth, C = twins.filtered_moments(H, Z, M, cls, ldos=True)
    ld_filt = C[nodes].copy()
    del C
    _log("BA-1M filtered done in %.0f s" % (time.time() - t0))
    np.savez(os.path.join(HERE, "ba1m_twins_oracle.npz"), probe_seed=PROBE_SEED, graph_seed=GRAPH_SEED,
             n=g.n, nnz=g.nnz, n_classes=len(cls), nodes=nodes, mu_pp_plain=pp_plain, mu_pp_smooth=pp_smooth,
             mu_full_filtered=mu_full, ldos_plain=ld_plain, ldos_filtered=ld_filt)


def make_rmat22() -> None:
    from oracle import big
    W = WORKLOADS["rmat22"]
    k, M = W.probes, W.moments
    n, s, d = W.graph(GRAPH_SEED)
    g = big.BigGraph(n, s, d)
    del s, d
    deg = np.diff(g.row_ptr())
    nodes = _pick_nodes(deg, 32, 96, 13)
    _log("R-MAT-22 ef16: n=%d nnz=%d; %d moments" % (g.n, g.nnz, M))
    t0 = time.time()
    pp, ld = g.moments(k, M, PROBE_SEED, rows=nodes)
    _log("R-MAT-22 done in %.0f s" % (time.time() - t0))
    hist = rc.histogram(pp.mean(axis=0), W.bins)[0]
    np.savez(os.path.join(HERE, "rmat22_oracle.npz"), probe_seed=PROBE_SEED, graph_seed=GRAPH_SEED, n=g.n,
             nnz=g.nnz, nodes=nodes, mu_pp=pp, ldos=ld, hist200=hist)


def make_rmat27() -> None:
    from oracle import big
    W = WORKLOADS["rmat27"]
    k, M = W.probes, W.moments
    n, s, d = W.graph(GRAPH_SEED)
    _log("R-MAT-27: edges generated; building")
    g = big.BigGraph(n, s, d)
    del s, d
    deg = np.diff(g.row_ptr())
    nodes = _pick_nodes(deg, 16, 48, 17)
    _log("R-MAT-27: n=%d nnz=%d; %d moments" % (g.n, g.nnz, M))
    t0 = time.time()
    pp, ld = g.moments(k, M, PROBE_SEED, rows=nodes)
    _log("R-MAT-27 done in %.0f s" % (time.time() - t0))
    np.savez(os.path.join(HERE, "rmat27_oracle.npz"), probe_seed=PROBE_SEED, graph_seed=GRAPH_SEED, n=g.n,
             nnz=g.nnz, nodes=nodes, node_degree=deg[nodes], mu_pp=pp, ldos=ld)


if __name__ == "__main__":
    jobs = {"ba1m": make_ba1m, "rmat22": make_rmat22, "rmat27": make_rmat27}
    for name in sys.argv[1:] or list(jobs):
        jobs[name]()
