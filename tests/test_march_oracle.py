"""Pins of the time-marching generator, the oracle's damped Newton iteration and
the oracle's network (forward, gradient, Adam) against closed forms, library
routines and brute force (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from synth.assemble import assemble_jacobian
from synth.learned import init_mlp_params, minibatch_orders, mlp_layer_shapes
from synth.march import ChannelMarch
from synth.mesh import StructuredMesh
from synth.nonlinear import SlabOperator, extrapolation_matrix, poiseuille_slab
from synth.radau import radau_right


@pytest.mark.parametrize("k", [1, 2])
def test_poiseuille_is_an_exact_slab_solution(k):
    """Steady Poiseuille flow with p = 8 nu U (L - x) / H^2 solves the slab equations exactly
    for a constant inflow (Q2 x P1disc represent it; convection vanishes)."""
    m = StructuredMesh((10, 4), (2.2, 0.41), k)
    op = SlabOperator(m, 1e-3, 0.01)
    X = poiseuille_slab(m, 0.3, 1e-3)
    F = op.residual(X, X[:m.n_vel], 0.37, amplitude=lambda t: 0.3)
    scale = np.abs(op.jacobian(X) @ X).max()
    assert np.abs(F).max() <= 1e-13 * scale
    # a wrong pressure level or amplitude is not a solution
    Y = X.copy()
    Y[m.n_vel:m.n_space] += 1e-3
    assert np.abs(op.residual(Y, X[:m.n_vel], 0.0, amplitude=lambda t: 0.3)).max() > 1e-9
    assert np.abs(op.residual(X, X[:m.n_vel], 0.0, amplitude=lambda t: 0.31)).max() > 1e-6


@pytest.mark.parametrize("k", [1, 3])
def test_slab_jacobian_equals_assembled_newton_matrix(k):
    m = StructuredMesh((6, 4), (2.2, 0.41), k)
    op = SlabOperator(m, 2e-3, 0.02)
    X = np.random.default_rng(3).standard_normal(m.n) * 0.2
    J1 = op.jacobian(X)
    J2 = assemble_jacobian(m, op.velocity_state(X), 2e-3, 0.02)
    assert (J1 != J2).nnz == 0 or abs(J1 - J2).max() <= 1e-15 * abs(J2).max()
    assert np.array_equal(J1.indptr, J2.indptr) and np.array_equal(J1.indices, J2.indices)


def test_slab_residual_derivative_is_the_jacobian():
    m = StructuredMesh((6, 4), (2.2, 0.41), 1)
    op = SlabOperator(m, 1e-3, 0.01)
    rng = np.random.default_rng(4)
    X = rng.standard_normal(m.n) * 0.2
    up = rng.standard_normal(m.n_vel) * 0.2
    d = rng.standard_normal(m.n)
    eps = 1e-6
    fd = (op.residual(X + eps * d, up, 0.1) - op.residual(X - eps * d, up, 0.1)) / (2 * eps)
    assert np.abs(fd - op.jacobian(X) @ d).max() <= 1e-8 * np.abs(fd).max()


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_extrapolation_reproduces_polynomials_of_degree_k(k):
    s, _ = radau_right(k)
    E = extrapolation_matrix(k)
    for deg in range(k + 1):
        old = s ** deg                  # p(t) = t^deg on the previous slab [0, 1]
        new = (1.0 + s) ** deg          # on the next slab [1, 2]
        np.testing.assert_allclose(E @ old, new, rtol=1e-12, atol=1e-12)
    if k == 1:
        np.testing.assert_allclose(E, [[-0.5, 1.5], [-1.5, 2.5]], atol=1e-14)


def test_oracle_newton_converges_quadratically():
    pr = ChannelMarch(shape=(8, 4), levels=2, k=1)
    X_prev = pr.initial_slab()
    # a poor start so that several Newton steps are needed; tight inner solves
    X, its_n, its_g, hist = oracle.newton_slab(lambda X: pr.residual(X, X_prev, 1), pr.hierarchy,
                                               X_prev + 0.2 * np.random.default_rng(0).standard_normal(pr.n),
                                               tol=1e-12, rtol=1e-12, atol=1e-14)
    assert hist[-1] < 1e-12 and its_n >= 3
    # quadratic convergence: ||F_{k+1}|| <= C ||F_k||^2 with a moderate C at every step
    ratios = [hist[i + 1] / hist[i] ** 2 for i in range(len(hist) - 1)]
    assert max(ratios) < 10.0, ratios
    np.testing.assert_array_less(np.diff(hist), 0.0)


def test_oracle_march_matches_direct_newton():
    """Each marched slab solves F = 0: the residual of every slab is below the tolerance, and
    a dense direct Newton solve from the same guess gives the same slab solution."""
    pr = ChannelMarch(shape=(8, 4), levels=2, k=1)
    Xs, counts = oracle.march(pr, 3)
    for n in range(1, 4):
        assert np.linalg.norm(pr.residual(Xs[n], Xs[n - 1], n)) < 1e-8
    # direct Newton with dense solves
    X = pr.extrapolate(Xs[2])
    for _ in range(8):
        F = pr.residual(X, Xs[2], 3)
        if np.linalg.norm(F) < 1e-12:
            break
        X = X + np.linalg.solve(pr.hierarchy(X)[-1].J.toarray(), -F)
    assert np.abs(X - Xs[3]).max() <= 1e-6 * np.abs(X).max()


# ---- network oracle ----------------------------------------------------------------------------

def _small_net(seed=0):
    shapes = mlp_layer_shapes(6, 5, 3, 4)
    p = init_mlp_params(6, 5, 3, 4, seed=seed).astype(np.float64)
    p += 0.05 * np.random.default_rng(seed).standard_normal(p.size)   # non-zero biases
    rng = np.random.default_rng(100 + seed)
    return shapes, p, rng.standard_normal((7, 6)), rng.standard_normal((7, 4))


def test_mlp_forward_by_hand():
    """One hidden unit: y = w2 tanh(w1 x + b1) + b2."""
    shapes = mlp_layer_shapes(1, 1, 1, 1)
    p = np.array([0.7, -0.2, 1.5, 0.3])
    _, y = omlp.forward(p, shapes, np.array([[0.4]]))
    assert abs(y[0, 0] - (1.5 * np.tanh(0.7 * 0.4 - 0.2) + 0.3)) < 1e-15


def test_mlp_gradient_equals_central_differences():
    shapes, p, X, T = _small_net()
    L, g = omlp.loss_and_grad(p, shapes, X, T)
    eps = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        fd[i] = (omlp.loss_and_grad(p + e, shapes, X, T)[0] - omlp.loss_and_grad(p - e, shapes, X, T)[0]) / (2 * eps)
    assert np.abs(fd - g).max() <= 1e-8 * np.abs(g).max()
    assert L == pytest.approx(np.mean((omlp.forward(p, shapes, X)[1] - T) ** 2), rel=1e-14)


def test_mlp_bf16_points_stay_within_rounding_bound():
    shapes, p, X, T = _small_net(1)
    _, y = omlp.forward(p, shapes, X)
    _, yb = omlp.forward(p, shapes, X, bf16_points=True)
    # inputs, weights and activations each carry a relative error <= 2^-8 (BF16 unit roundoff 2^-9 doubled
    # for the products); four layers: 4 * 3 * 2^-8 ~ 5e-2 as a normwise bound
    assert np.linalg.norm(yb - y) <= 5e-2 * np.linalg.norm(y)


def test_adam_first_step_closed_form():
    """With zero moments, Adam's first step moves every parameter by lr g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    th, g = rng.standard_normal(50), rng.standard_normal(50)
    new, m, v = omlp.adam_step(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=4e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=4e-15)


def test_adam_minimises_a_quadratic():
    th = np.array([3.0, -2.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        th, m, v = omlp.adam_step(th, m, v, 2.0 * (th - np.array([1.0, 0.5])), t, lr=1e-2)
    np.testing.assert_allclose(th, [1.0, 0.5], atol=1e-3)


def test_minibatch_orders_are_permutations():
    o = minibatch_orders(1000, 3, seed=2)
    assert o.shape == (3, 1000) and o.dtype == np.int32
    for row in o:
        assert np.array_equal(np.sort(row), np.arange(1000))
    assert not np.array_equal(o[0], o[1])
