"""Pins of the MLP / importance-sampling oracle (learned-proposal form).

* gradients against central finite differences of the loss (FP64);
* closed forms: a one-neuron linear network, silu at known points, and the
  silu derivative against finite differences;
* Adam: the first step moves each parameter by lr * sign(g) (bias correction);
* importance sampling: the exact expectation of sum_j w_j t(q_j) over the
  proposal equals the mesh average, for any proposal with full support;
* inverse CDF against a brute-force scan;
* BF16 rounding: ties to even at known points and torch's CPU bfloat16 cast.
"""

import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    n_in, width, depth = 5, 7, 3
    theta = mlp.init_params(rng, n_in, width, depth)
    theta[: theta.size // 3] += 0.3 * rng.standard_normal(theta.size // 3)
    X = rng.standard_normal((11, n_in))
    t = rng.standard_normal(11)
    loss, g = mlp.loss_and_grad(theta, X, t, n_in, width, depth)
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        lp, _ = mlp.loss_and_grad(theta + e, X, t, n_in, width, depth)
        lm, _ = mlp.loss_and_grad(theta - e, X, t, n_in, width, depth)
        num[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-7 * max(1.0, np.max(np.abs(g)))


def test_one_neuron_linear_closed_form():
    # depth 0: y = w.x + b ; L = mean (y - t)^2 ; dL/dw = 2/B sum (y - t) x
    theta = np.array([0.5, -1.0, 0.25])           # W [1,2], b [1]
    X = np.array([[1.0, 2.0], [3.0, -1.0]])
    t = np.array([0.0, 1.0])
    loss, g = mlp.loss_and_grad(theta, X, t, 2, 4, 0)
    y = X @ theta[:2] + theta[2]
    r = y - t
    assert abs(loss - np.mean(r ** 2)) < 1e-15
    assert np.allclose(g, np.concatenate([2 * (r @ X) / 2, [2 * r.sum() / 2]]), atol=1e-15)


def test_silu_values_and_derivative():
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.silu(np.array([1.0]))[0] - 1.0 / (1.0 + np.exp(-1.0))) < 1e-16
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_prime(z))) < 1e-9


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g), atol=1e-15)


def test_importance_sampling_expectation_is_exact():
    rng = np.random.default_rng(1)
    N = 37
    t = rng.exponential(size=N)
    p = rng.uniform(0.1, 1.0, size=N)
    p /= p.sum()
    S = 5
    # expectation over S iid draws: S * sum_q p(q) * t(q) / (N S p(q)) = mean(t)
    w_single = mlp.is_weights(p, np.arange(N), N)      # weight of each q if drawn (S=N here)
    exp_val = S * np.sum(p * t * (w_single * N / S))
    assert abs(exp_val - t.mean()) < 1e-12


def test_inverse_cdf_brute_force():
    rng = np.random.default_rng(2)
    p = rng.uniform(0, 1, size=20)
    p[3] = 0.0
    u = rng.uniform(0, 1, size=200)
    got = mlp.inverse_cdf(p, u)
    c = np.cumsum(p)
    for uj, gj in zip(u, got):
        j = 0
        while c[j] <= uj * c[-1]:
            j += 1
        assert gj == j
        assert p[gj] > 0


def test_round_bf16_ties_and_library():
    """Round to nearest even at 8 significant bits; agrees with torch's CPU bfloat16 cast."""
    torch = pytest.importorskip("torch")
    one = 1.0
    assert mlp.round_bf16(one + 2.0 ** -8) == 1.0                      # tie -> even (down)
    assert mlp.round_bf16(one + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (up)
    assert mlp.round_bf16(one + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mlp.round_bf16(-3.0) == -3.0 and mlp.round_bf16(0.0) == 0.0
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(50_000) * 10.0 ** rng.integers(-6, 6, 50_000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(mlp.round_bf16(x), ref)


def test_operand_rounding_reaches_every_product():
    """With BF16-exact parameters and inputs the first product is exact; rounding the
    operands changes the gradient of every layer (it reaches the backward products)."""
    rng = np.random.default_rng(4)
    n_in, width, depth, B = 5, 7, 2, 9
    theta = mlp.round_bf16(mlp.init_params(rng, n_in, width, depth))
    X = mlp.round_bf16(rng.standard_normal((B, n_in)))
    t = rng.standard_normal(B)
    y0, z0 = mlp.forward(theta, X, n_in, width, depth)
    y1, z1 = mlp.forward(theta, X, n_in, width, depth, operand=mlp.round_bf16)
    assert np.allclose(z0[0], z1[0], rtol=0, atol=1e-15)
    _, g0 = mlp.loss_and_grad(theta, X, t, n_in, width, depth)
    _, g1 = mlp.loss_and_grad(theta, X, t, n_in, width, depth, operand=mlp.round_bf16)
    off = 0
    for o, i in mlp.layer_shapes(n_in, width, depth):
        dw0, dw1 = g0[off:off + o * i], g1[off:off + o * i]
        assert np.max(np.abs(dw0 - dw1)) > 0
        assert np.max(np.abs(dw0 - dw1)) < 2e-2 * np.max(np.abs(dw0))
        off += o * i + o
