"""Seeded initial parameters for the control-variate MLP (an input to
training, shared by the GPU trainer and the oracle's tests).

Layout of the flat fp32 vector: [W1 (5 x 128, row-major in x out), b1 (128),
W2 (128 x 128), b2 (128), W3 (128 x n_out), b3 (n_out)].  Weights are
He-uniform (bound sqrt(6 / fan_in)), biases zero, from numpy's seeded PCG64.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 5
WIDTH = 128


def init_params(seed: int, n_out: int = 64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in [(N_FEAT, WIDTH), (WIDTH, WIDTH), (WIDTH, n_out)]:
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=(fan_in, fan_out)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
