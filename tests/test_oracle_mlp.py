"""Pins of the FP64 oracle of the learned self-collision screen (a small
SiLU multilayer perceptron with a Huber loss): closed-form special cases of
the forward pass and central finite differences of its gradient."""
import math

import numpy as np
import pytest

import oracle


def silu(z):
    return z / (1.0 + math.exp(-z))


def layout(D, H):
    sizes = [H * D, H, H * H, H, H * H, H, H, 1]
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    out, o = {}, 0
    for n, s in zip(names, sizes):
        out[n] = slice(o, o + s)
        o += s
    return out, o


def test_num_params_matches_the_workload_network():
    assert oracle.mlp_num_params(7, 256) == 133_889
    assert oracle.mlp_num_params(3, 4) == layout(3, 4)[1]


def test_forward_closed_form_constant_layers():
    """W1 = W2 = W3 = 0: every hidden unit of layer l equals silu(b_l[i]), so
    y = b4 + sum_i W4[i] silu(b3[i]) whatever the input."""
    D, H = 7, 5
    sl, P = layout(D, H)
    p = np.zeros(P)
    rng = np.random.default_rng(0)
    p[sl["b1"]] = rng.normal(size=H)
    p[sl["b2"]] = rng.normal(size=H)
    p[sl["b3"]] = rng.normal(size=H)
    p[sl["W4"]] = rng.normal(size=H)
    p[sl["b4"]] = 0.3
    x = rng.normal(size=(4, D))
    want = 0.3 + sum(p[sl["W4"]][i] * silu(p[sl["b3"]][i]) for i in range(H))
    np.testing.assert_allclose(oracle.mlp_forward(D, H, p, x), want, atol=1e-14)


def test_forward_scalar_chain():
    """H = 1: y = b4 + w4 silu(w3 silu(w2 silu(w1 . x + b1) + b2) + b3)."""
    D, H = 3, 1
    sl, P = layout(D, H)
    p = np.arange(1, P + 1, dtype=float) * 0.1 - 0.35
    x = np.array([[0.2, -0.7, 0.4]])
    w1 = p[sl["W1"]]
    a1 = silu(w1 @ x[0] + p[sl["b1"]][0])
    a2 = silu(p[sl["W2"]][0] * a1 + p[sl["b2"]][0])
    a3 = silu(p[sl["W3"]][0] * a2 + p[sl["b3"]][0])
    want = p[sl["b4"]][0] + p[sl["W4"]][0] * a3
    np.testing.assert_allclose(oracle.mlp_forward(D, H, p, x), want, atol=1e-15)


def test_loss_huber_regimes_and_target_clipping():
    """All weights zero, b4 = 0: y = 0, so the loss is the mean Huber of the
    clipped targets: quadratic inside the threshold, linear outside."""
    D, H = 2, 3
    _, P = layout(D, H)
    p = np.zeros(P)
    x = np.zeros((4, D))
    t = np.array([0.01, -0.04, 0.2, 9.0])            # 9.0 is clipped to 0.5
    d = 0.05
    want = np.mean([0.5 * 0.01 ** 2, 0.5 * 0.04 ** 2, d * (0.2 - d / 2), d * (0.5 - d / 2)])
    assert abs(oracle.mlp_loss(D, H, p, x, t, d, -0.3, 0.5) - want) < 1e-15


@pytest.mark.parametrize("D,H,n", [(7, 8, 16), (3, 5, 9)])
def test_gradient_central_finite_differences_all_params(D, H, n):
    rng = np.random.default_rng(D * 10 + H)
    _, P = layout(D, H)
    p = rng.normal(size=P) * 0.5
    x = rng.uniform(-1, 1, size=(n, D))
    t = rng.uniform(-0.4, 0.6, size=n)           # some targets clipped
    loss, g = oracle.mlp_loss_grad(D, H, p, x, t)
    assert abs(loss - oracle.mlp_loss(D, H, p, x, t)) < 1e-15
    h = 1e-6
    fd = np.empty(P)
    for k in range(P):
        e = np.zeros(P)
        e[k] = h
        fd[k] = (oracle.mlp_loss(D, H, p + e, x, t) - oracle.mlp_loss(D, H, p - e, x, t)) / (2 * h)
    rel = np.linalg.norm(fd - g) / np.linalg.norm(g)
    assert rel < 1e-6, rel


def test_gradient_finite_differences_full_size_sampled():
    D, H, n = 7, 256, 8
    sl, P = layout(D, H)
    rng = np.random.default_rng(5)
    p = rng.normal(size=P) * np.sqrt(1.0 / 256)
    p[sl["W1"]] = rng.normal(size=H * D) * np.sqrt(1.0 / D)
    x = rng.uniform(-1, 1, size=(n, D))
    t = rng.uniform(-0.2, 0.4, size=n)
    _, g = oracle.mlp_loss_grad(D, H, p, x, t)
    idx = np.concatenate([rng.choice(np.arange(s.start, s.stop), 8, replace=False) if s.stop - s.start > 8
                          else np.arange(s.start, s.stop) for s in sl.values()])
    h = 1e-6
    for k in idx:
        e = np.zeros(P)
        e[k] = h
        fd = (oracle.mlp_loss(D, H, p + e, x, t) - oracle.mlp_loss(D, H, p - e, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, np.abs(g).max()), (k, fd, g[k])
