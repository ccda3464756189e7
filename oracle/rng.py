"""Probe vectors for the stochastic trace / diagonal estimators (Sec. 3.1,
eq. probe_trace and eq. probe_diag): entries i.i.d. with mean 0, variance 1.

The paper's analysis uses standard normal entries; its experiments use
"Hadamard" (+/-1) probes.  Both are provided here:

* Rademacher: z_ij = +1 or -1 from the top bit of a SplitMix64 output.
* Gaussian:   Box-Muller on two 53-bit uniforms, rounded to fp32 (the GPU
  stores probe blocks in fp32, so the fp32 value *is* the probe).

Counter-based definition (one generator, implemented independently here and in
the GPU library from SplitMix64's published definition -- Steele, Lea & Flood,
OOPSLA 2014): output n >= 1 of the stream seeded with s is
``mix(s + n * 0x9E3779B97F4A7C15)`` with the SplitMix64 finalizer ``mix``.

* probe j's stream key is output j+1 of the stream seeded with ``seed``;
* Rademacher entry (j, i) uses output i+1 of probe j's stream;
* Gaussian entry (j, i) uses outputs 2i+1 and 2i+2.

Node index i is the compacted node id (after isolated nodes are dropped).
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> int:
    """Output n (1-based) of the SplitMix64 stream seeded with `seed` (Python ints)."""
    z = (seed + n * GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_np(seed: int, n: np.ndarray) -> np.ndarray:
    """Vectorised `splitmix64` over an array of 1-based output indices."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + np.asarray(n, dtype=np.uint64) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def probe_key(seed: int, j: int) -> int:
    return splitmix64(seed, j + 1)


def rademacher(n_nodes: int, n_probes: int, seed: int) -> np.ndarray:
    """[n_nodes][n_probes] float64 array of +/-1."""
    Z = np.empty((n_nodes, n_probes), np.float64)
    idx = np.arange(1, n_nodes + 1, dtype=np.uint64)
    for j in range(n_probes):
        b = splitmix64_np(probe_key(seed, j), idx)
        Z[:, j] = np.where((b >> np.uint64(63)) != 0, -1.0, 1.0)
    return Z


def gaussian(n_nodes: int, n_probes: int, seed: int) -> np.ndarray:
    """[n_nodes][n_probes] standard normal probes, values rounded to fp32."""
    Z = np.empty((n_nodes, n_probes), np.float64)
    i = np.arange(n_nodes, dtype=np.uint64)
    for j in range(n_probes):
        key = probe_key(seed, j)
        b1 = splitmix64_np(key, np.uint64(2) * i + np.uint64(1))
        b2 = splitmix64_np(key, np.uint64(2) * i + np.uint64(2))
        u1 = ((b1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53
        u2 = (b2 >> np.uint64(11)).astype(np.float64) * 2.0**-53
        g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        Z[:, j] = g.astype(np.float32).astype(np.float64)
    return Z


def probes(n_nodes: int, n_probes: int, seed: int, kind: str = "rademacher") -> np.ndarray:
    if kind == "rademacher":
        return rademacher(n_nodes, n_probes, seed)
    if kind == "gaussian":
        return gaussian(n_nodes, n_probes, seed)
    raise ValueError(kind)


def rademacher_at(nodes: np.ndarray, n_probes: int, seed: int) -> np.ndarray:
    """Rows `nodes` of the Rademacher probe block: [len(nodes)][n_probes]
    (same definition as :func:`rademacher`, evaluated at selected node ids)."""
    idx = np.asarray(nodes, dtype=np.uint64) + np.uint64(1)
    Z = np.empty((idx.size, n_probes), np.float64)
    for j in range(n_probes):
        b = splitmix64_np(probe_key(seed, j), idx)
        Z[:, j] = np.where((b >> np.uint64(63)) != 0, -1.0, 1.0)
    return Z
