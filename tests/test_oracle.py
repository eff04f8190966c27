"""Pins of the FP64 oracle against what the paper and the mathematics fix:
brute-force dense operators on tiny meshes, the local-residual invariant of a
patch solve, special cases (one cell, one level, M = I, M = J^-1) and the
minimal-residual property of GMRES."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import build_problem
from synth.problems import build_hierarchy


def tiny(shape=(2, 2), levels=1, k=1, seed=3, nu=1e-2):
    lvls = build_hierarchy(d=len(shape), shape=shape, lengths=(0.8, 0.41, 0.41)[: len(shape)],
                           levels=levels, k=k, nu=nu, tau=0.01, U=0.3, seed=seed)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(lvls[-1].n)
    d = rng.standard_normal(lvls[-1].n)
    return lvls, b, d


def dense_vanka_operator(J, cell_dofs, omega):
    """D = omega P^-1 sum_K E_K J_K^-1 R_K built from explicit dense E_K and J_K."""
    Jd = J.toarray()
    n = Jd.shape[0]
    D = np.zeros((n, n))
    p = np.zeros(n)
    for dofs in cell_dofs:
        E = np.zeros((n, len(dofs)))
        E[dofs, np.arange(len(dofs))] = 1.0
        JK = E.T @ Jd @ E
        D += E @ np.linalg.solve(JK, E.T)
        p += E.sum(axis=1)
    return omega * D / p[:, None]


def test_patch_matrix_is_principal_submatrix():
    lvls, _, _ = tiny((3, 2))
    L = lvls[-1]
    Jd = L.J.toarray()
    for K in range(L.mesh.n_cells):
        dofs = L.cell_dofs[K]
        np.testing.assert_array_equal(oracle.patch_matrix(L.J, dofs), Jd[np.ix_(dofs, dofs)])


def test_patch_inverse_identity():
    lvls, _, _ = tiny((3, 2), k=2)
    L = lvls[-1]
    JK = oracle.patch_matrices(L.J, L.cell_dofs)
    A = oracle.invert_patches(JK)
    cond = np.linalg.cond(JK)
    for K in range(len(A)):
        err = np.abs(JK[K] @ A[K] - np.eye(JK.shape[1])).max()
        assert err <= 1e-13 * cond[K]


@pytest.mark.parametrize("shape", [(1, 1), (2, 1), (2, 2)])
@pytest.mark.parametrize("order", ["sequential", "coloured"])
def test_additive_sweep_equals_dense_operator(shape, order):
    lvls, b, d = tiny(shape)
    L = lvls[-1]
    A, p = oracle.setup_level(L.J, L.cell_dofs)
    omega = 0.7
    want = d + dense_vanka_operator(L.J, L.cell_dofs, omega) @ (b - L.J @ d)
    for f in (oracle.additive_sweep, oracle.additive_sweep_loop):
        got = f(L.J, A, L.cell_dofs, b, d, omega, order, L.colours)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    got = oracle.additive_sweep_correction(L.J, A, L.cell_dofs, p, b, d, omega, order, L.colours)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_additive_sequential_equals_coloured():
    lvls, b, d = tiny((6, 4))
    L = lvls[-1]
    A, _ = oracle.setup_level(L.J, L.cell_dofs)
    s = oracle.additive_sweep(L.J, A, L.cell_dofs, b, d, 0.7, "sequential")
    c = oracle.additive_sweep(L.J, A, L.cell_dofs, b, d, 0.7, "coloured", L.colours)
    assert np.abs(s - c).max() <= 1e-13 * np.abs(s).max()


def test_one_cell_exact_solve():
    """On a one-cell mesh J_K = J, so one sweep with omega = 1 solves J d = b."""
    lvls, b, d = tiny((1, 1))
    L = lvls[-1]
    A, _ = oracle.setup_level(L.J, L.cell_dofs)
    for mode in ("additive", "multiplicative"):
        x = oracle.smooth(L.J, A, L.cell_dofs, None if mode == "multiplicative" else
                          oracle.multiplicity(L.cell_dofs, L.n), b, d, 1, 1.0, mode, "sequential")
        assert np.linalg.norm(L.J @ x - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("omega", [1.0, 0.7])
def test_local_residual_after_patch_solve(omega):
    """Updating only K: (b - J d')[dofs_K] = (1 - omega)(b - J d)[dofs_K]."""
    lvls, b, d = tiny((3, 3))
    L = lvls[-1]
    A, _ = oracle.setup_level(L.J, L.cell_dofs)
    for K in [0, 4, 8]:
        one = np.array([L.cell_dofs[K]])
        dn = oracle.multiplicative_sweep(L.J, A[K:K + 1], one, b, d, omega, "sequential")
        r0 = (b - L.J @ d)[one[0]]
        r1 = (b - L.J @ dn)[one[0]]
        np.testing.assert_allclose(r1, (1 - omega) * r0, rtol=0, atol=1e-12 * np.abs(r0).max())


def test_multiplicative_sequential_against_loop_by_hand():
    """Sequential overwriting = d_K += omega J_K^-1 R_K(b - J d) cell after cell, with
    dense algebra; and the last cell's local residual vanishes for omega = 1."""
    lvls, b, d = tiny((3, 2))
    L = lvls[-1]
    A, _ = oracle.setup_level(L.J, L.cell_dofs)
    Jd = L.J.toarray()
    x = d.copy()
    for dofs in L.cell_dofs:
        r = b - Jd @ x
        x[dofs] += 0.7 * np.linalg.solve(Jd[np.ix_(dofs, dofs)], r[dofs])
    got = oracle.multiplicative_sweep(L.J, A, L.cell_dofs, b, d, 0.7, "sequential")
    np.testing.assert_allclose(got, x, rtol=1e-12, atol=1e-12 * np.abs(x).max())
    g1 = oracle.multiplicative_sweep(L.J, A, L.cell_dofs, b, d, 1.0, "sequential")
    last = L.cell_dofs[-1]
    assert np.abs((b - L.J @ g1)[last]).max() <= 1e-11 * np.abs(b).max()


def test_multiplicative_coloured_one_cell_per_colour_is_sequential():
    lvls, b, d = tiny((2, 2))
    L = lvls[-1]
    assert sorted(L.colours) == [0, 1, 2, 3]
    A, _ = oracle.setup_level(L.J, L.cell_dofs)
    s = oracle.multiplicative_sweep(L.J, A, L.cell_dofs, b, d, 0.7, "sequential")
    c = oracle.multiplicative_sweep(L.J, A, L.cell_dofs, b, d, 0.7, "coloured", L.colours)
    np.testing.assert_allclose(c, s, rtol=0, atol=1e-14 * np.abs(s).max())


def test_multiplicative_coloured_is_jacobi_within_colour():
    """Dense form: for each colour c, d += omega sum_{K in c} E_K J_K^-1 R_K (b - J d)."""
    lvls, b, d = tiny((4, 4))
    L = lvls[-1]
    A, _ = oracle.setup_level(L.J, L.cell_dofs)
    Jd = L.J.toarray()
    x = d.copy()
    for c in range(4):
        r = b - Jd @ x
        upd = np.zeros_like(x)
        for K in np.nonzero(L.colours == c)[0]:
            dofs = L.cell_dofs[K]
            upd[dofs] += np.linalg.solve(Jd[np.ix_(dofs, dofs)], r[dofs])
        x = x + 0.7 * upd
    got = oracle.multiplicative_sweep(L.J, A, L.cell_dofs, b, d, 0.7, "coloured", L.colours)
    np.testing.assert_allclose(got, x, rtol=1e-12, atol=1e-12 * np.abs(x).max())


def test_vcycle_single_level_is_direct_solve():
    lvls, b, _ = tiny((3, 2), levels=1)
    H = oracle.OracleHierarchy(lvls)
    x = oracle.vcycle(H, b)
    assert np.linalg.norm(lvls[0].J @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_vcycle_two_levels_dense():
    """Two levels, nu1 = nu2 = 1: V = S-post(d0 + P J0^-1 R (b - J d0)), d0 = S-pre(0),
    with the smoother as the dense affine map d -> d + D (b - J d)."""
    lvls, b, _ = tiny((4, 2), levels=2)
    H = oracle.OracleHierarchy(lvls, omega=0.7, mode="additive", order="coloured")
    L1, L0 = lvls[1], lvls[0]
    J1, J0 = L1.J.toarray(), L0.J.toarray()
    D = dense_vanka_operator(L1.J, L1.cell_dofs, 0.7)
    P = L1.P.toarray()
    d = D @ b
    d = d + P @ np.linalg.solve(J0, P.T @ (b - J1 @ d))
    d = d + D @ (b - J1 @ d)
    got = oracle.vcycle(H, b, 1, 1)
    np.testing.assert_allclose(got, d, rtol=1e-10, atol=1e-10 * np.abs(d).max())
    # nu = 0: pure coarse-grid correction P J0^-1 R b
    got0 = oracle.vcycle(H, b, 0, 0)
    want0 = P @ np.linalg.solve(J0, P.T @ b)
    np.testing.assert_allclose(got0, want0, rtol=1e-10, atol=1e-10 * np.abs(want0).max())


def test_vcycle_linear():
    lvls, b, d = tiny((4, 4), levels=2)
    H = oracle.OracleHierarchy(lvls)
    v1, v2 = oracle.vcycle(H, b), oracle.vcycle(H, d)
    v3 = oracle.vcycle(H, 2.5 * b + d)
    assert np.abs(v3 - 2.5 * v1 - v2).max() <= 1e-12 * np.abs(v3).max()


def test_gmres_minimal_residual_property():
    """With M = I, the j-th iterate minimises ||b - J x|| over the Krylov space K_j(J, b):
    brute force by least squares on an orthonormalised Krylov basis."""
    rng = np.random.default_rng(7)
    n = 40
    J = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    _, its, hist, conv, _ = oracle.gmres(J, b, lambda v: v, restart=60, max_iter=25, rtol=1e-30)
    assert its == 25
    Kb = [b / np.linalg.norm(b)]
    for j in range(1, 26):
        Q, _ = np.linalg.qr(np.array(Kb).T)
        y, *_ = np.linalg.lstsq(J @ Q, b, rcond=None)
        best = np.linalg.norm(b - J @ Q @ y)
        assert abs(hist[j] - best) <= 1e-9 * np.linalg.norm(b), j
        Kb.append(J @ Kb[-1])
        Kb[-1] /= np.linalg.norm(Kb[-1])


def test_gmres_identity_precond_full_space_exact():
    rng = np.random.default_rng(8)
    n = 30
    J = np.eye(n) + 0.5 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, its, hist, conv, rel = oracle.gmres(J, b, lambda v: v, restart=n, max_iter=n, rtol=1e-12)
    assert its <= n and conv
    np.testing.assert_allclose(J @ x, b, atol=1e-10)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def test_gmres_exact_preconditioner_one_step():
    rng = np.random.default_rng(9)
    n = 25
    J = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    Jinv = np.linalg.inv(J)
    x, its, *_ = oracle.gmres(J, b, lambda v: Jinv @ v, restart=30, max_iter=30, rtol=1e-10)
    assert its == 1


def test_gmres_restart_and_zero_rhs():
    rng = np.random.default_rng(10)
    n = 60
    J = np.eye(n) * 2 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, its, hist, conv, rel = oracle.gmres(J, b, lambda v: v, restart=5, max_iter=200, rtol=1e-10)
    assert conv and rel <= 1e-10 and its > 5
    x0, its0, *_ = oracle.gmres(J, np.zeros(n), lambda v: v)
    assert its0 == 0 and np.all(x0 == 0)


def test_gmres_vcycle_cfg0_matches_direct_solve(cfg0):
    H = oracle.OracleHierarchy(cfg0.levels)
    J = cfg0.finest.J
    x, its, hist, conv, rel = oracle.gmres(J, cfg0.b, lambda v: oracle.vcycle(H, v, 2, 2))
    assert conv and rel <= 1e-8
    # history estimate equals the true residual at the end
    assert abs(hist[-1] - np.linalg.norm(cfg0.b - J @ x)) <= 1e-10 * np.linalg.norm(cfg0.b)
    assert np.all(np.diff(hist) <= 0)
    xs = sp.linalg.spsolve(J.tocsc(), cfg0.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-5


def test_k_robustness_small():
    """Sec. 4: GMRES counts do not grow with k; on one mesh they differ by at most 1 for k = 1..3."""
    counts = []
    for k in (1, 2, 3):
        P = build_problem("channel2d_44x8_k1", k=k, shape=(22, 4), levels=2)
        H = oracle.OracleHierarchy(P.levels)
        _, its, *_ = oracle.gmres(P.finest.J, P.b, lambda v: oracle.vcycle(H, v, 2, 2))
        counts.append(its)
    assert max(counts) - min(counts) <= 1, counts


def test_bf16_rounding_rne():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -3.140625, 1e-30])
    r = oracle.round_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0   # tie between 1 and 1+2^-7: even mantissa -> 1.0
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7                  # above the tie rounds up
    assert r[3] == 1.0                            # below
    assert r[4] == -3.140625
    assert abs(r[5] - 1e-30) <= 2 ** -8 * 1e-30
    y = np.random.default_rng(0).standard_normal(1000)
    assert np.all(np.abs(oracle.round_bf16(y) - y) <= 2 ** -8 * np.abs(y))
    assert np.all(np.abs(oracle.round_f32(y) - y) <= 2 ** -24 * np.abs(y))
