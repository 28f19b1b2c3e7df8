"""Pins of the fp64 selector-network reference (oracle/mlp.py) and of the
library's host-side selector helpers.  No GPU.

The reference is checked against things other than itself: central finite
differences of the loss (the backward pass), networks whose output is known
in closed form (forward pass and flat parameter layout), and the closed form
of Adam's first steps.
"""
import numpy as np
import pytest

from oracle import mlp


def _problem(k, b, seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(k, seed) + rng.normal(0, 0.05, mlp.param_count(k))
    x = rng.normal(0, 1, (b, 16))
    t = rng.normal(0, 1, (b, k))
    m = (rng.random((b, k)) < 0.7).astype(np.float64)
    m[0, :] = 0.0  # one sample without labels
    return p, x, t, m


def test_param_count_matches_layout():
    # 16*64 + 64 + 64*64 + 64 + 65*64 + 65
    assert mlp.param_count(65) == 9473
    assert mlp.param_count(1) == 1024 + 64 + 4096 + 64 + 64 + 1


@pytest.mark.parametrize("k,b,seed", [(3, 5, 0), (65, 4, 1), (1, 7, 2)])
def test_gradient_matches_central_differences(k, b, seed):
    p, x, t, m = _problem(k, b, seed)
    _, g = mlp.loss_and_grad(p, k, x, t, m)
    rng = np.random.default_rng(seed + 100)
    # every bias of the output layer plus a random sample of the other entries
    idx = np.concatenate([np.arange(mlp.param_count(k) - k, mlp.param_count(k)),
                          rng.choice(mlp.param_count(k) - k, 200, replace=False)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, k, x, t, m) - mlp.loss(p - e, k, x, t, m)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_loss_matches_value_of_gradient_call():
    p, x, t, m = _problem(5, 6, 3)
    L, _ = mlp.loss_and_grad(p, 5, x, t, m)
    assert L == pytest.approx(mlp.loss(p, 5, x, t, m), rel=1e-12)


def test_forward_closed_form_and_layout():
    # Hidden unit i of layer 1 copies feature i (i < 16) through the ReLU
    # (features are positive), layer 2 copies unit i, output k sums features
    # 0..k with weight (k+1) and adds bias 10 k.
    k = 4
    W1 = np.zeros((64, 16))
    W1[np.arange(16), np.arange(16)] = 1.0
    W2 = np.eye(64)
    W3 = np.zeros((k, 64))
    for j in range(k):
        W3[j, : j + 1] = j + 1
    b3 = 10.0 * np.arange(k)
    p = mlp.pack(W1, np.zeros(64), W2, np.zeros(64), W3, b3)
    x = np.arange(1, 17, dtype=np.float64)[None, :] * np.array([[1.0], [2.0]])
    y, _ = mlp.forward(p, k, x)
    for s in range(2):
        for j in range(k):
            assert y[s, j] == (j + 1) * x[s, : j + 1].sum() + 10.0 * j


def test_relu_blocks_negative_units():
    k = 2
    W1 = np.zeros((64, 16))
    W1[0, 0] = 1.0
    b1 = np.zeros(64)
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    W3 = np.zeros((k, 64))
    W3[:, 0] = 1.0
    p = mlp.pack(W1, b1, W2, np.zeros(64), W3, np.zeros(k))
    x = np.zeros((2, 16))
    x[0, 0] = 3.0
    x[1, 0] = -3.0  # clipped to zero by the first ReLU
    y, _ = mlp.forward(p, k, x)
    assert y[0].tolist() == [3.0, 3.0] and y[1].tolist() == [0.0, 0.0]


def test_loss_closed_form_and_zero_weights():
    k = 2
    p = mlp.pack(np.zeros((64, 16)), np.zeros(64), np.zeros((64, 64)), np.zeros(64), np.zeros((k, 64)),
                 np.array([1.0, -2.0]))
    x = np.zeros((2, 16))
    t = np.array([[0.0, 0.0], [3.0, 1.0]])
    m = np.array([[1.0, 1.0], [1.0, 0.0]])
    # sample 0: ((1-0)^2 + (-2-0)^2) / 2 = 2.5; sample 1: (1-3)^2 / 1 = 4; mean 3.25
    assert mlp.loss(p, k, x, t, m) == pytest.approx(3.25, rel=1e-15)
    L, g = mlp.loss_and_grad(p, k, x, t, np.zeros_like(m))
    assert L == 0.0 and not g.any()


def test_adam_first_steps_closed_form():
    # With zero moments, bias correction makes the first step
    # -lr * g / (|g| + eps); a constant gradient keeps that step size.
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    lr, eps = 0.01, 1e-8
    p1, m1, v1 = mlp.adam_step(p, np.zeros(4), np.zeros(4), g, 1, lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    p2, _, _ = mlp.adam_step(p1, m1, v1, g, 2, lr, eps=eps)
    assert np.allclose(p2 - p1, p1 - p, rtol=0, atol=1e-12)


def test_selector_cells_grid():
    jp = pytest.importorskip("paper_2002_12459_amd")
    f = [0.0] * 16
    f[7], f[12], f[14] = np.log1p(400.0), np.log1p(90.0), np.log1p(19.0)
    d1, d2 = jp.selector_cells(f)
    assert len(d1) == len(d2) == 65
    assert d1[64] is None and d2[64] is None
    # Delta1 geometric from 2 to the larger y maximum, Delta2 from 1 to the x maximum
    for i in range(8):
        for j in range(8):
            a = 2.0 * (400.0 / 2.0) ** (i / 7.0)
            b = 19.0 ** (j / 7.0)
            assert abs(d1[8 * i + j] - a) <= 0.5 + 1e-3 and abs(d2[8 * i + j] - b) <= 0.5 + 1e-3
    assert d1[0] == 2 and d1[63] == 400 and d2[0] == 1 and d2[63] == 19
    # degenerate instance: no degrees above 1
    d1, d2 = jp.selector_cells([0.0] * 16)
    assert set(d1[:64]) == {2} and set(d2[:64]) == {1}


def test_mlp_param_count_export():
    jp = pytest.importorskip("paper_2002_12459_amd")
    assert jp.mlp_param_count(65) == mlp.param_count(65)
    assert jp.mlp_param_count(1) == mlp.param_count(1)
