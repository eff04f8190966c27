"""Seeded random inputs of the learned initial guess (a project extension): the
initial network weights and the minibatch orders of training.  Both the FP64
oracle and the GPU trainer take these arrays as inputs; this module holds no
network arithmetic.
"""
import numpy as np

# network of the learned guess: inputs = the patch values of the two previous slab
# solutions (2 n_K), three hidden tanh layers of width 128, output = n_K
WIDTH, N_HIDDEN = 128, 3


def mlp_layer_shapes(n_in, width, n_hidden, n_out):
    return [(width, n_in)] + [(width, width)] * (n_hidden - 1) + [(n_out, width)]


def init_mlp_params(n_in, width=WIDTH, n_hidden=N_HIDDEN, n_out=None, seed=0):
    """Packed FP32 parameters [W_1, b_1, ...]: W_l uniform in +-sqrt(6 / (fan_in + fan_out))
    (Glorot), biases zero, the output layer scaled by 0.1."""
    n_out = n_in if n_out is None else n_out
    rng = np.random.default_rng(5000 + seed)
    shapes = mlp_layer_shapes(n_in, width, n_hidden, n_out)
    parts = []
    for l, (o, i) in enumerate(shapes):
        a = np.sqrt(6.0 / (o + i)) * (0.1 if l == len(shapes) - 1 else 1.0)
        parts.append(rng.uniform(-a, a, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def minibatch_orders(n_samples, epochs, seed=0):
    """One random permutation of the samples per epoch (int32 [epochs, n_samples])."""
    rng = np.random.default_rng(6000 + seed)
    return np.stack([rng.permutation(n_samples) for _ in range(epochs)]).astype(np.int32)
