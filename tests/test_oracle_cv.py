"""Pins for the control-variate oracle (CPU only).  The learned control
variate is not in the paper: these pin the features, MLP gradient and Adam
update to their mathematical definitions (parity unpinned by the paper)."""
import numpy as np
import pytest

import synthgraph as sg
from synthgraph.mlp_init import init_params
from oracle import graph as og
from oracle import cv


def test_features_bruteforce():
    for gen in (sg.erdos_renyi(80, 0.08, seed=1), sg.barabasi_albert(60, 2, seed=4, twin_pairs=5)):
        g = og.build_csr(*gen)
        assert np.allclose(cv.raw_features(g), cv.raw_features_bruteforce(g))


def test_features_textbook():
    g = og.build_csr(*sg.complete(6))           # every node: d=5, clustering 1, no 2-hop
    f = cv.raw_features(g)
    assert np.allclose(f, [[5, 5, 5, 1.0, 0]] * 6)
    g = og.build_csr(*sg.star(4))               # hub: 2-hop 0; leaf: 2-hop = other leaves
    f = cv.raw_features(g)
    assert f[0].tolist() == [4, 1, 1, 0.0, 0] and f[1].tolist() == [1, 4, 4, 0.0, 3]
    g = og.build_csr(*sg.cycle(9))              # 2-hop count 2, no triangles
    assert np.allclose(cv.raw_features(g), [[2, 2, 2, 0.0, 2]] * 9)


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(0)
    p = init_params(3, n_out=8).astype(np.float64)
    p[cv.n_params(8) - 8:] += rng.normal(size=8) * 0.1  # non-zero output bias
    x = rng.normal(size=(12, 5))
    t = rng.normal(size=(12, 8))
    loss, grad = cv.mse_grad(p, x, t, n_out=8)
    assert loss == pytest.approx(cv.mse(p, x, t, n_out=8))
    h = 1e-6
    idx = rng.choice(p.size, 60, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (cv.mse(p + e, x, t, 8) - cv.mse(p - e, x, t, 8)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 + 1e-5 * abs(fd)


def test_adam_first_step_is_signed_lr():
    # after one step from zero moments, m_hat / sqrt(v_hat) = g / |g|
    g = np.array([0.5, -2.0, 1e-3, -1e-4])
    p, m, v = cv.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, t=1, lr=0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-4)


def test_param_count():
    assert cv.n_params() == 25536
    assert init_params(0).size == 25536 and init_params(0).dtype == np.float32


def test_mlp_forward_soft_threshold_closed_form():
    """The forward pass against a closed form: with the first layer splitting
    each feature into relu(x) and relu(-x), the second shifting both by -1/2
    before its ReLU and the third taking their difference through a matrix
    C, the network computes S(x) C + b3 with S the soft threshold
    sign(x) max(|x| - 1/2, 0).  A dropped ReLU or bias, or a transposed or
    misplaced block of the flat parameter vector, changes the result."""
    rng = np.random.default_rng(3)
    n_out = 8
    W1, b1, W2, b2, W3, b3 = (np.zeros(s) for s in
                              [(5, 128), (128,), (128, 128), (128,), (128, n_out), (n_out,)])
    C = rng.normal(size=(5, n_out))
    for k in range(5):
        W1[k, k], W1[k, 5 + k] = 1.0, -1.0
        W2[k, k], W2[5 + k, 5 + k] = 1.0, 1.0
        W3[k], W3[5 + k] = C[k], -C[k]
    b2[:10] = -0.5
    b3[:] = rng.normal(size=n_out)
    x = rng.normal(scale=1.5, size=(40, 5))
    soft = np.sign(x) * np.maximum(np.abs(x) - 0.5, 0.0)
    got = cv.forward(cv.pack([W1, b1, W2, b2, W3, b3]), x, n_out=n_out)
    assert np.allclose(got, soft @ C + b3, rtol=0, atol=1e-12)
