"""Seeded synthetic graph generators (edge lists) shared by the GPU library's
tests, the CPU oracle's tests and the benchmark.

Only input generation lives here: none of the spectral-density arithmetic.
The generators are C (``gen.c``, built with gcc and OpenMP into
``libsynthgraph.so`` next to this file) and deterministic for a given seed,
whatever the thread count.

Every generator returns ``(n_nodes, src, dst)`` with ``src``/``dst`` int32
numpy arrays: an undirected edge list over ids ``[0, n_nodes)`` that may hold
duplicates, self-loops (R-MAT, WS) and isolated nodes.  The graph builder of
either side turns it into the symmetric, simple graph the method works on.

Workload recipes (sizes and model parameters) live in :mod:`synthgraph.workloads`.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynthgraph.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libsynthgraph.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        p = ctypes.c_void_p
        lib.sg_er.argtypes = [i64, dbl, u64, i64, p, p]
        lib.sg_er.restype = i64
        lib.sg_sbm.argtypes = [i64, i32, dbl, dbl, u64, i64, p, p]
        lib.sg_sbm.restype = i64
        lib.sg_ba.argtypes = [i64, i32, i64, u64, i64, p, p]
        lib.sg_ba.restype = i64
        lib.sg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, i64, p, p]
        lib.sg_rmat.restype = None
        lib.sg_ws.argtypes = [i64, i32, dbl, u64, i64, p, p]
        lib.sg_ws.restype = i64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _grow(fn, expected: float):
    """Run a generator that reports its edge count; retry once if the buffer
    was too small (the second run reproduces the first exactly)."""
    cap = int(expected + 8.0 * math.sqrt(max(expected, 1.0)) + 1024)
    src = np.empty(cap, np.int32)
    dst = np.empty(cap, np.int32)
    m = fn(cap, src, dst)
    if m > cap:
        src = np.empty(m, np.int32)
        dst = np.empty(m, np.int32)
        m2 = fn(m, src, dst)
        assert m2 == m
    return src[:m].copy(), dst[:m].copy()


def erdos_renyi(n: int, p: float, seed: int):
    """G(n, p): each pair {u, v}, u != v, present independently with prob. p."""
    lib = _load()
    exp = p * n * (n - 1) / 2.0
    src, dst = _grow(lambda cap, s, d: lib.sg_er(n, p, seed, cap, _ptr(s), _ptr(d)), exp)
    return n, src, dst


def sbm(n: int, p_in: float, p_out: float, seed: int, nblocks: int = 4):
    """Stochastic block model: `nblocks` equal blocks, p_in within, p_out across."""
    lib = _load()
    b = n / nblocks
    exp = nblocks * p_in * b * (b - 1) / 2.0 + p_out * (n * n - nblocks * b * b) / 2.0
    src, dst = _grow(
        lambda cap, s, d: lib.sg_sbm(n, nblocks, p_in, p_out, seed, cap, _ptr(s), _ptr(d)), exp
    )
    return n, src, dst


def barabasi_albert(n: int, m: int, seed: int, twin_pairs: int = 0):
    """Preferential attachment from an (m+1)-clique, plus `twin_pairs` pairs of
    leaves (ids n + 2q, n + 2q + 1) attached to a shared hub drawn uniformly
    from the first n nodes.  Total node count n + 2*twin_pairs."""
    lib = _load()
    ne = m * (m + 1) // 2 + (n - m - 1) * m + 2 * twin_pairs
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    got = lib.sg_ba(n, m, twin_pairs, seed, ne, _ptr(src), _ptr(dst))
    if got != ne:
        raise ValueError("barabasi_albert: bad arguments (n=%d, m=%d)" % (n, m))
    return n + 2 * twin_pairs, src, dst


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19, n_mod: int = 0):
    """R-MAT with 2^scale * edge_factor samples.  With n_mod > 0 the ids are
    reduced modulo n_mod and the node count is n_mod, else 2^scale."""
    lib = _load()
    ne = (1 << scale) * edge_factor
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    lib.sg_rmat(scale, ne, a, b, c, seed, n_mod, _ptr(src), _ptr(dst))
    return (n_mod if n_mod > 0 else (1 << scale)), src, dst


def watts_strogatz(n: int, k: int, p: float, seed: int):
    """Ring lattice (k/2 neighbours per side) with each edge rewired w.p. p."""
    lib = _load()
    ne = n * (k // 2)
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    got = lib.sg_ws(n, k, p, seed, ne, _ptr(src), _ptr(dst))
    assert got == ne
    return n, src, dst


# Small deterministic graphs with textbook spectra (used by the pins).
def cycle(n: int):
    u = np.arange(n, dtype=np.int32)
    return n, u, ((u + 1) % n).astype(np.int32)


def path(n: int):
    u = np.arange(n - 1, dtype=np.int32)
    return n, u, (u + 1).astype(np.int32)


def complete(n: int):
    iu, ju = np.triu_indices(n, 1)
    return n, iu.astype(np.int32), ju.astype(np.int32)


def star(s: int):
    """Hub 0 with s leaves."""
    return s + 1, np.zeros(s, np.int32), np.arange(1, s + 1, dtype=np.int32)


def complete_bipartite(a: int, b: int):
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return a + b, u.ravel().astype(np.int32), v.ravel().astype(np.int32)


def friendship(k: int):
    """Windmill of k triangles on hub 0: blade q is the adjacent pair
    (2q+1, 2q+2), both joined to the hub."""
    q = np.arange(k, dtype=np.int32)
    a, b = 2 * q + 1, 2 * q + 2
    hub = np.zeros(k, np.int32)
    return 2 * k + 1, np.concatenate([a, a, b]), np.concatenate([b, hub, hub])


def plant_adjacent_pairs(n: int, src, dst, pairs: int, seed: int, hubs=(1, 2, 3)):
    """Append `pairs` new adjacent node pairs (ids n + 2q, n + 2q + 1); pair q
    is joined, both nodes, to h distinct nodes drawn uniformly from [0, n),
    h cycling through `hubs`.  Returns (n + 2 * pairs, src, dst)."""
    rng = np.random.default_rng(seed)
    s_add, d_add = [], []
    for q in range(pairs):
        u, v = n + 2 * q, n + 2 * q + 1
        h = hubs[q % len(hubs)]
        targets = rng.choice(n, size=h, replace=False)
        s_add += [u] + [u] * h + [v] * h
        d_add += [v] + list(targets) + list(targets)
    src = np.concatenate([np.asarray(src, np.int32), np.asarray(s_add, np.int32)])
    dst = np.concatenate([np.asarray(dst, np.int32), np.asarray(d_add, np.int32)])
    return n + 2 * pairs, src, dst


def grid2d(nx: int, ny: int):
    """nx x ny lattice, node (i, j) = i * ny + j, 4-neighbour edges."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    node = (i * ny + j).astype(np.int32)
    s = np.concatenate([node[:-1, :].ravel(), node[:, :-1].ravel()])
    d = np.concatenate([node[1:, :].ravel(), node[:, 1:].ravel()])
    return nx * ny, s.astype(np.int32), d.astype(np.int32)
