"""Pins of the input generator: closed forms, exact reproduction properties and
the DoF counts the paper prints."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle  # noqa: E402
from synth import StructuredMesh, dg_time_matrices, radau_right, build_problem, hierarchy_shapes
from synth.assemble import element_matrices, local_pattern, volume_rule, tensor_basis
from synth.transfer import prolongation, inject_nodes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _ev(expr):
    return eval(expr, {"sqrt": np.sqrt})


@pytest.mark.parametrize("k", [0, 1, 2])
def test_radau_nodes_weights_closed_form(k):
    g = _load("radau_iia.json")
    s, w = radau_right(k)
    np.testing.assert_allclose(s, [_ev(e) for e in g["nodes"][str(k)]], rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, [_ev(e) for e in g["weights"][str(k)]], rtol=0, atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("z", [-0.5, -3.0, 2j, -10.0 + 1j])
def test_dg_radau_is_radau_iia(k, z):
    """dG(k) on y' = lambda y gives y(t_n) = R(z) y(t_{n-1}), z = tau lambda."""
    g = _load("radau_iia.json")["stability"][str(k)]
    _, w, Kt, c0 = dg_time_matrices(k)
    Y = np.linalg.solve(Kt - z * np.diag(w), c0.astype(complex))
    R = np.polyval(g["num"][::-1], z) / np.polyval(g["den"][::-1], z)
    assert abs(Y[-1] - R) < 1e-12 * max(1.0, abs(R))


def test_dg0_is_implicit_euler():
    _, w, Kt, c0 = dg_time_matrices(0)
    assert Kt.shape == (1, 1) and Kt[0, 0] == 1.0 and w[0] == 1.0 and c0[0] == 1.0


@pytest.mark.parametrize("shape,k,nK", [((4, 2), 1, 42), ((4, 2), 2, 63), ((4, 2), 3, 84),
                                        ((2, 2, 2), 1, 170)])
def test_patch_width(shape, k, nK):
    m = StructuredMesh(shape, (1.0,) * len(shape), k)
    assert m.n_K == nK and m.cell_dofs().shape == (m.n_cells, nK)


def test_dof_counts_closed_form():
    def count(shape, k):
        d = len(shape)
        return (k + 1) * (d * int(np.prod([2 * n + 1 for n in shape])) + (d + 1) * int(np.prod(shape)))
    assert StructuredMesh((44, 8), (2.2, 0.41), 1).n == count((44, 8), 1) == 8164
    assert StructuredMesh((176, 32), (2.2, 0.41), 2).n == count((176, 32), 2) == 188358
    assert StructuredMesh((100, 16, 16), (2.5, 0.41, 0.41), 1).n == count((100, 16, 16), 1) == 1518134


def test_paper_dof_tables_scale_with_k_plus_1():
    """Tables 4.1-4.3 print DoFs per slab = (k+1) x a spatial count; so does the generator."""
    g = _load("paper_tables.json")
    for tab in ("table_4_1_dofs", "table_4_2_dofs"):
        base = g[tab]["0"]
        for k, v in g[tab].items():
            assert v == (int(k) + 1) * base
    assert g["table_4_3_dofs_k1"] == g["table_4_2_dofs"]["1"]
    for k in range(5):
        assert StructuredMesh((6, 2), (1, 1), k).n == (k + 1) * StructuredMesh((6, 2), (1, 1), 0).n


def test_hierarchy_shapes():
    assert hierarchy_shapes((44, 8), 3) == [(11, 2), (22, 4), (44, 8)]
    assert hierarchy_shapes((176, 32), 5)[0] == (11, 2)
    assert hierarchy_shapes((100, 16, 16), 4) == [(25, 2, 2), (25, 4, 4), (50, 8, 8), (100, 16, 16)]


def test_colouring_is_dof_disjoint():
    for shape in [(6, 4), (3, 3, 2)]:
        m = StructuredMesh(shape, (1.0,) * len(shape), 1)
        cd, col = m.cell_dofs(), m.colours()
        assert col.max() + 1 == m.n_colours
        for c in range(m.n_colours):
            dofs = cd[col == c].ravel()
            assert len(np.unique(dofs)) == len(dofs)


def test_multiplicity_closed_form_2d():
    """p: interior vertex 4, boundary vertex 2, corner 1, interior edge midpoint 2,
    boundary midpoint 1, cell centre 1, pressure 1."""
    m = StructuredMesh((4, 3), (1, 1), 0)
    p = oracle.multiplicity(m.cell_dofs(), m.n)   # the oracle's count, pinned by the closed form
    ni = m.node_index()
    vx = p[: m.n_vel: 2]
    for node, (ix, iy) in enumerate(ni):
        bx = ix in (0, m.node_shape[0] - 1)
        by = iy in (0, m.node_shape[1] - 1)
        if ix % 2 == 0 and iy % 2 == 0:
            want = 1 if (bx and by) else (2 if (bx or by) else 4)
        elif ix % 2 == 1 and iy % 2 == 1:
            want = 1
        else:
            on_line_boundary = (iy % 2 == 0 and by) or (ix % 2 == 0 and bx)
            want = 1 if on_line_boundary else 2
        assert vx[node] == want, (ix, iy)
    assert np.all(p[m.n_vel:] == 1)


def _poly_q2(x):
    out = np.ones(x.shape[0])
    for i in range(x.shape[1]):
        c = [1.0 + i, -0.5 * (i + 1), 0.75]
        out *= c[0] + c[1] * x[:, i] + c[2] * x[:, i] ** 2
    return out


@pytest.mark.parametrize("fine", [(4, 2), (4, 4, 2), (6, 2, 2)])
def test_prolongation_reproduces_q2_and_p1(fine):
    d = len(fine)
    fm = StructuredMesh(fine, (2.0, 1.0, 0.5)[:d], 1)
    cshape = tuple(n // 2 if n % 2 == 0 and n >= 4 else n for n in fine)
    cm = StructuredMesh(cshape, fm.lengths, 1)
    P = prolongation(cm, fm)
    assert P.shape == (fm.n, cm.n)
    # velocity: a product of quadratics per direction is in Q2
    uc = np.zeros(cm.n)
    want = np.zeros(fm.n)
    xc, xf = cm.node_coords(), fm.node_coords()
    for a in range(2):
        for c in range(d):
            uc[a * cm.n_space + np.arange(cm.n_nodes) * d + c] = (c + 1 + a) * _poly_q2(xc)
            want[a * fm.n_space + np.arange(fm.n_nodes) * d + c] = (c + 1 + a) * _poly_q2(xf)
    # pressure: a global linear field; coefficients in each cell's {1, x^, y^} basis
    coef = np.array([0.3, -1.2, 0.7, 2.0])[: d + 1]

    def pres(m):
        centres = (m.cell_index() + 0.5) * np.array(m.h)
        c0 = coef[0] + centres @ coef[1:]
        slopes = np.broadcast_to(coef[1:][None, :] * np.array(m.h)[None, :] / 2.0, (m.n_cells, d))
        return np.concatenate([c0[:, None], slopes], axis=1).ravel()
    for a in range(2):
        uc[a * cm.n_space + cm.n_vel: (a + 1) * cm.n_space] = pres(cm)
        want[a * fm.n_space + fm.n_vel: (a + 1) * fm.n_space] = pres(fm)
    np.testing.assert_allclose(P @ uc, want, rtol=0, atol=1e-12)


def test_prolongation_1d_quarter_weights():
    from synth.transfer import prolong_1d
    P1 = prolong_1d(1, True).toarray()
    np.testing.assert_allclose(P1[1], [3 / 8, 3 / 4, -1 / 8])
    np.testing.assert_allclose(P1[3], [-1 / 8, 3 / 4, 3 / 8])
    np.testing.assert_allclose(P1.sum(axis=1), 1.0)


def test_injection_nodes_coincide():
    fm = StructuredMesh((8, 4), (2.0, 1.0), 1)
    cm = StructuredMesh((4, 2), (2.0, 1.0), 1)
    np.testing.assert_allclose(fm.node_coords()[inject_nodes(cm, fm)], cm.node_coords())


def test_element_integrals():
    m = StructuredMesh((3, 2), (0.6, 0.5), 0)
    pts, w = volume_rule(m)
    phi, dphi = tensor_basis(m, pts)
    M = np.einsum("q,qn,qm->nm", w, phi, phi)
    assert abs(M.sum() - np.prod(m.h)) < 1e-14
    S = np.einsum("q,qni,qmi->nm", w, dphi, dphi)
    np.testing.assert_allclose(S.sum(axis=1), 0.0, atol=1e-12)
    # (v . grad f, phi_n) for f = x, v = (1, 0) equals int phi_n
    xn = m.local_node_offsets()[:, 0] * m.h[0] / 2.0
    conv = np.einsum("q,qn,qm->nm", w, phi, dphi[:, :, 0]) @ xn
    np.testing.assert_allclose(conv, M.sum(axis=1), atol=1e-14)


def test_jacobian_structure(cfg0):
    L = cfg0.levels[0]
    m = L.mesh
    J = L.J.toarray()
    ns, nv = m.n_space, m.n_vel
    _, w, Kt, _ = dg_time_matrices(m.k)
    tau = cfg0.params["tau"]
    for a in range(m.n_time):
        pa = slice(a * ns + nv, (a + 1) * ns)
        va = slice(a * ns, a * ns + nv)
        assert np.all(J[pa, pa] == 0.0)
        np.testing.assert_allclose(J[pa, va], J[va, pa].T, rtol=0, atol=1e-15)
        for b in range(m.n_time):
            if a != b:
                vb = slice(b * ns, b * ns + nv)
                assert np.all(J[va, b * ns + nv:(b + 1) * ns] == 0.0)
                Mref = J[vb, vb] * 0  # shape holder
                # velocity mass recovered from the cross-time block
                Mv = J[va, vb] / Kt[a, b]
                assert np.allclose(Mv, Mv.T, atol=1e-15)
                assert abs(Mv[::2, ::2].sum() - np.prod(m.lengths)) < 1e-12


def test_jacobian_zero_state_symmetric():
    """With v^m = 0 the same-time velocity block minus Kt[a,a] M is symmetric (Stokes + Nitsche)."""
    from synth.assemble import assemble_jacobian
    m = StructuredMesh((3, 2), (0.9, 0.41), 1)
    V = np.zeros((m.n_time, m.n_nodes, m.d))
    J = assemble_jacobian(m, V, 1e-2, 0.01).toarray()
    _, _, Kt, _ = dg_time_matrices(1)
    ns, nv = m.n_space, m.n_vel
    Mv = J[0:nv, ns:ns + nv] / Kt[0, 1]
    for a in range(2):
        blk = J[a * ns:a * ns + nv, a * ns:a * ns + nv] - Kt[a, a] * Mv
        np.testing.assert_allclose(blk, blk.T, atol=1e-14)


def test_nnz_counts_match_structure(cfg0):
    assert [L.J.nnz for L in cfg0.levels] == [22908, 89100, 351372]
    pat = local_pattern(cfg0.levels[0].mesh)
    assert pat.shape == (42, 42)


# ---- velocity degree r = 4: (Q4)^2 x P3disc, the element of the paper's 2D study (Sec. 4) ----

@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_q4_patch_width_and_counts(k):
    """n_K = (k + 1)(2 * 25 + 10) = 60 (k + 1); spatial DoFs 2 (4 nx + 1)(4 ny + 1) + 10 nx ny."""
    m = StructuredMesh((5, 3), (1.0, 0.6), k, r=4)
    assert m.n_K == 60 * (k + 1) and m.cell_dofs().shape == (15, m.n_K)
    assert m.n == (k + 1) * (2 * 21 * 13 + 10 * 15)
    assert np.array_equal(np.unique(m.cell_dofs()), np.arange(m.n))  # every DoF is in some patch


def test_q4_lagrange_basis_and_gauss_rule():
    from synth.assemble import _lagrange_1d, gauss_rule_01
    nodes = np.arange(5) / 4
    v, dv = _lagrange_1d(nodes, 4)
    np.testing.assert_allclose(v, np.eye(5), atol=1e-15)               # nodal
    s = np.random.default_rng(3).uniform(0, 1, 7)
    v, dv = _lagrange_1d(s, 4)
    np.testing.assert_allclose(v.sum(axis=1), 1.0, atol=1e-14)          # reproduces 1 ...
    np.testing.assert_allclose(dv.sum(axis=1), 0.0, atol=1e-12)
    np.testing.assert_allclose(v @ nodes ** 4, s ** 4, atol=1e-14)       # ... and s^4
    np.testing.assert_allclose(dv @ nodes ** 4, 4 * s ** 3, atol=1e-12)
    g, w = gauss_rule_01(4)                                             # 6 points: exact to degree 11
    assert len(g) == 6
    for p in range(12):
        assert abs(w @ g ** p - 1.0 / (p + 1)) < 1e-15


def test_q4_prolongation_reproduces_q4_and_p3():
    """Nested spaces: a degree-4 velocity field and a cubic pressure field pass unchanged."""
    from synth.assemble import pressure_basis
    c = StructuredMesh((3, 2), (1.5, 1.0), 0, r=4)
    f = StructuredMesh((6, 4), (1.5, 1.0), 0, r=4)
    P = prolongation(c, f)
    u = lambda x: x[:, 0] ** 4 - 2 * x[:, 0] ** 2 * x[:, 1] ** 2 + x[:, 1] ** 3 + 0.5
    vc = np.zeros(c.n)
    vc[0:c.n_vel:2] = u(c.node_coords())
    vc[1:c.n_vel:2] = -u(c.node_coords())
    vf = P @ vc
    np.testing.assert_allclose(vf[0:f.n_vel:2], u(f.node_coords()), atol=1e-13)
    np.testing.assert_allclose(vf[1:f.n_vel:2], -u(f.node_coords()), atol=1e-13)

    def coeffs(m, p):
        """Per-cell P3 coefficients of p, fitted on sample points of each cell."""
        s = np.random.default_rng(1).uniform(0, 1, size=(30, 2))
        B = pressure_basis(s, 4)
        ci = m.cell_index()
        return np.concatenate([np.linalg.lstsq(B, p((ci[K] + s) * np.array(m.h)), rcond=None)[0]
                               for K in range(m.n_cells)])
    p = lambda X: X[:, 0] ** 3 - X[:, 0] * X[:, 1] ** 2 + 2 * X[:, 1] - 1
    pc = np.zeros(c.n)
    pc[c.n_vel:] = coeffs(c, p)
    np.testing.assert_allclose((P @ pc)[f.n_vel:], coeffs(f, p), atol=1e-12)
    np.testing.assert_allclose(f.node_coords()[inject_nodes(c, f)], c.node_coords())


def test_q4_element_integrals():
    m = StructuredMesh((3, 2), (0.6, 0.5), 0, r=4)
    pts, w = volume_rule(m)
    phi, dphi = tensor_basis(m, pts)
    M = np.einsum("q,qn,qm->nm", w, phi, phi)
    assert abs(M.sum() - np.prod(m.h)) < 1e-14
    S = np.einsum("q,qni,qmi->nm", w, dphi, dphi)
    np.testing.assert_allclose(S.sum(axis=1), 0.0, atol=1e-11)
    # int grad(x^2 y^2) . grad(x^2 y^2) over the cell [0, hx] x [0, hy], from the nodal interpolant
    hx, hy = m.h
    xn = m.local_node_offsets() * np.array(m.h) / 4.0
    g = xn[:, 0] ** 2 * xn[:, 1] ** 2
    exact = 4 * (hx ** 3 / 3) * (hy ** 5 / 5) + 4 * (hx ** 5 / 5) * (hy ** 3 / 3)
    assert abs(g @ S @ g - exact) < 1e-14


def test_q4_jacobian_zero_state_symmetric():
    """As for Q2: with v^m = 0 the same-time velocity block minus Kt[a,a] M is symmetric, and the
    pressure rows are the negated transposed divergence columns."""
    from synth.assemble import assemble_jacobian
    m = StructuredMesh((3, 2), (0.9, 0.41), 1, r=4)
    J = assemble_jacobian(m, np.zeros((m.n_time, m.n_nodes, m.d)), 1e-2, 0.01).toarray()
    _, _, Kt, _ = dg_time_matrices(1)
    ns, nv = m.n_space, m.n_vel
    Mv = J[0:nv, ns:ns + nv] / Kt[0, 1]
    assert abs(Mv[::2, ::2].sum() - np.prod(m.lengths)) < 1e-12
    for a in range(2):
        blk = J[a * ns:a * ns + nv, a * ns:a * ns + nv] - Kt[a, a] * Mv
        np.testing.assert_allclose(blk, blk.T, atol=1e-13)
        pa, va = slice(a * ns + nv, (a + 1) * ns), slice(a * ns, a * ns + nv)
        assert np.all(J[pa, pa] == 0.0)
        np.testing.assert_allclose(J[pa, va], J[va, pa].T, atol=1e-15)
