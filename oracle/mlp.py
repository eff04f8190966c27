"""FP64 multilayer perceptron, loss gradient and Adam step: the oracle of the
learned initial guess (a project extension; the paper has no learned part).

Network: n_in -> width (tanh) -> ... (n_hidden hidden layers of `width`, tanh)
-> n_out (linear).  Parameters are one packed vector, layer by layer: W_l
(out x in, row-major) then b_l.  Loss over a batch of B samples:
    L = 1 / (B n_out) * sum_{m, j} (y_mj - t_mj)^2.
The gradient is the chain rule written out layer by layer (reverse mode).
Adam (Kingma & Ba, Algorithm 1): with g the gradient at step t,
    m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
    theta -= lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).

`bf16_points=True` rounds (RNE to BF16) at the points where a BF16 kernel
stores: the inputs, the weights used in products, every hidden activation and
every back-propagated pre-activation gradient; arithmetic stays FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from .precision import round_bf16


def layer_shapes(n_in, width, n_hidden, n_out):
    return [(width, n_in)] + [(width, width)] * (n_hidden - 1) + [(n_out, width)]


def n_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(params, shapes):
    out, p = [], 0
    for o, i in shapes:
        W = params[p:p + o * i].reshape(o, i)
        p += o * i
        b = params[p:p + o]
        p += o
        out.append((W, b))
    return out


def forward(params, shapes, X, bf16_points=False):
    """Return (activations [a_0 = X, a_1, ..., a_L-1], y)."""
    rnd = round_bf16 if bf16_points else (lambda a: a)
    layers = unpack(np.asarray(params, dtype=np.float64), shapes)
    a = rnd(np.asarray(X, dtype=np.float64))
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = a @ rnd(W).T + b
        if l + 1 < len(layers):
            a = rnd(np.tanh(z))
            acts.append(a)
        else:
            return acts, z
    raise ValueError("empty network")


def loss_and_grad(params, shapes, X, T, bf16_points=False):
    """Mean squared error and its gradient with respect to the packed parameters."""
    rnd = round_bf16 if bf16_points else (lambda a: a)
    layers = unpack(np.asarray(params, dtype=np.float64), shapes)
    acts, y = forward(params, shapes, X, bf16_points)
    B, n_out = y.shape
    diff = y - T
    loss = float(np.sum(diff * diff) / (B * n_out))
    dz = rnd(2.0 * diff / (B * n_out))
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_prev = acts[l]
        grads[l] = (dz.T @ a_prev, dz.sum(axis=0))
        if l > 0:
            da = dz @ rnd(W)
            dz = rnd(da * (1.0 - a_prev * a_prev))
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(params, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
