"""FP64 oracle of the learned q-proposal: MLP, loss, gradients, Adam, sampler weights.

The learned-proposal form replaces the uniform sum over the q mesh by an
importance-sampled estimate whose proposal comes from a small multilayer
perceptron trained on integrand samples of the plain rate sum (Transport
Methods, electron lifetime: the per-(q, mode) terms of 1/tau).  This module is
the plain definition the GPU kernels are checked against:

* network: x -> z_1 = W_1 x + b_1, a_1 = silu(z_1), ..., z_L = W_L a_{L-1} + b_L
  (linear output), silu(z) = z / (1 + e^{-z});
* parameters packed layer by layer as W_l [out, in] (row major) then b_l [out];
* loss: mean squared error over the batch, L = (1/B) sum_b (y_b - t_b)^2;
* gradients by the chain rule (written out below, no autodiff library);
* Adam (Kingma & Ba, 2015) with bias correction;
* importance-sampling weights: with proposal p over the N_q mesh points and S
  draws, w_j = 1 / (N_q S p(q_j)) makes sum_j w_j t(q_j) an unbiased estimate of
  (1/N_q) sum_q t(q).

Pinned in tests/test_oracle_mlp.py by central finite differences, closed forms
of one-neuron networks, and the exact expectation of the estimator.
"""

import numpy as np


def layer_shapes(n_in, width, depth, n_out=1):
    """[(out, in), ...] for depth hidden layers of the given width."""
    dims = [n_in] + [width] * depth + [n_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def n_params(n_in, width, depth, n_out=1):
    return sum(o * i + o for o, i in layer_shapes(n_in, width, depth, n_out))


def unpack(theta, n_in, width, depth, n_out=1):
    """Views (W_l, b_l) of the packed parameter vector."""
    out = []
    off = 0
    for o, i in layer_shapes(n_in, width, depth, n_out):
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def init_params(rng, n_in, width, depth, n_out=1):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights, zero biases (the usual default)."""
    parts = []
    for o, i in layer_shapes(n_in, width, depth, n_out):
        lim = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def round_bf16(x):
    """Nearest bfloat16 value of each entry (8 significant bits, ties to even).

    The entries are first taken to float32, the storage of the BF16 network's
    operands; x = m 2^e with m in [0.5, 1) is rounded at 2^(e-8) by numpy's
    round-half-to-even.  Used to state the BF16 arithmetic exactly: operands
    of every matrix product rounded to BF16, products and sums exact.
    """
    f = np.asarray(x, dtype=np.float32).astype(np.float64)
    m, e = np.frexp(f)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def _ident(x):
    return x


def forward(theta, X, n_in, width, depth, n_out=1, operand=None):
    """Network output [B, n_out] and the pre-activations of every layer.

    ``operand`` (default: none) is applied to both inputs of every matrix
    product, e.g. ``round_bf16`` for the BF16 arithmetic.
    """
    op = operand or _ident
    layers = unpack(np.asarray(theta, dtype=np.float64), n_in, width, depth, n_out)
    a = np.asarray(X, dtype=np.float64)
    zs = []
    for li, (W, b) in enumerate(layers):
        z = op(a) @ op(W).T + b
        zs.append(z)
        a = z if li == len(layers) - 1 else silu(z)
    return a, zs


def loss_and_grad(theta, X, t, n_in, width, depth, n_out=1, operand=None):
    """MSE loss and its gradient with respect to the packed parameters.

    ``operand`` as in ``forward``: applied to both inputs of every matrix
    product of the forward and backward passes.
    """
    op = operand or _ident
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64).reshape(X.shape[0], n_out)
    layers = unpack(np.asarray(theta, dtype=np.float64), n_in, width, depth, n_out)
    acts = [X]
    zs = []
    a = X
    for li, (W, b) in enumerate(layers):
        z = op(a) @ op(W).T + b
        zs.append(z)
        a = z if li == len(layers) - 1 else silu(z)
        acts.append(a)
    B = X.shape[0]
    y = acts[-1]
    loss = float(np.sum((y - t) ** 2) / B)
    grads = []
    dz = 2.0 * (y - t) / B                     # dL/dz_L (linear output)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        dW = op(dz).T @ op(acts[li])           # [out, in]
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if li > 0:
            da = op(dz) @ op(W)                # dL/da_{l-1}
            dz = da * silu_prime(zs[li - 1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counter t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def is_weights(p, q_idx, n_q):
    """w_j = 1 / (N_q S p(q_j)) for S draws q_idx from the normalised proposal p."""
    p = np.asarray(p, dtype=np.float64)
    S = len(q_idx)
    return 1.0 / (n_q * S * p[np.asarray(q_idx)])


def inverse_cdf(p_unnorm, u):
    """Index j with CDF[j-1] <= u*total < CDF[j] for each uniform u in [0, 1)."""
    c = np.cumsum(np.asarray(p_unnorm, dtype=np.float64))
    return np.searchsorted(c, np.asarray(u) * c[-1], side="right")


def init_params_philox(seed, n_in, width, depth, n_out=1):
    """The library's deterministic initialisation: parameter j of the packed vector is a
    weight (2 u_j - 1) / sqrt(in_l), u_j element j of the Philox uniform stream (seed, 0)
    (``oracle.rng``), or a zero bias."""
    from .rng import uniform
    n = n_params(n_in, width, depth, n_out)
    u = uniform(seed, 0, n)
    theta = np.zeros(n)
    off = 0
    for o, i in layer_shapes(n_in, width, depth, n_out):
        theta[off:off + o * i] = (2.0 * u[off:off + o * i] - 1.0) / np.sqrt(i)
        off += o * i + o
    return theta


def training_set(terms, dweights, d_threshold, c_frac, max_samples, seed):
    """Training samples of the proposal network from the method's own terms.

    The network models the coupling part of the integrand: entries (state, q, nu)
    with D > d_threshold * max_{q, nu} D of their state are selected; an entry is
    kept when its Philox uniform (seed, flat index (state N_q + q) nModes + nu) is
    below min(1, max_samples / n_selected); its target is ln(T / D + c) with
    c = c_frac * mean over the selected entries of T / D.
    Returns (state, q, nu, y, c), entries in flat-index order.
    """
    from .rng import uniform
    T = np.asarray(terms, dtype=np.float64)
    D = np.asarray(dweights, dtype=np.float64)
    ns = T.shape[0]
    dmax = D.reshape(ns, -1).max(axis=1)
    sel = D > d_threshold * dmax[:, None, None]
    flat = np.flatnonzero(sel.ravel())
    ratio = T.ravel()[flat] / D.ravel()[flat]
    c = c_frac * ratio.mean() if flat.size else 0.0
    p_keep = min(1.0, max_samples / flat.size) if flat.size else 0.0
    u = uniform(seed, 0, T.size)[flat] if flat.size else np.zeros(0)
    keep = u < p_keep
    flat, ratio = flat[keep], ratio[keep]
    st, rem = np.divmod(flat, T.shape[1] * T.shape[2])
    q, nu = np.divmod(rem, T.shape[2])
    return st, q, nu, np.log(ratio + c), c
