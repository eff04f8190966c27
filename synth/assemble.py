"""Newton Jacobian of the dG(k) slab system on one mesh level (Sec. 2 Eq. 2.1,
2.2; Sec. 3 Eq. 3.2, 3.3).

The operator is the one of the variational problem: time derivative plus the
upwind jump (time matrix Kt of `radau.py`), the linearised convection
(v^m . grad) dv + (dv . grad) v^m, viscosity nu (grad v, grad psi), the
pressure coupling and Nitsche's weak Dirichlet terms with gamma_1 = gamma_2 = 35
on Gamma_D (inflow x = 0 and the walls); the outflow x = L_x is do-nothing.

Readings of the printed formulas (all generator-side):
  * rows are test functions, columns trial functions;
  * the Nitsche consistency and symmetry terms are those of A_h and B_GammaD
    (both with a minus sign), the penalty uses h of the cell normal to the face;
  * the continuity rows are negated, so that each slab block is exactly
    [D  B^T; B  0] with B^T[(n,c), q] = -(pi_q, d_c phi_n) + <pi_q, phi_n n_c>_GammaD;
  * time integrals use the (k+1)-point right Radau rule of the Lagrange nodes,
    so spatial operators are diagonal in time and the blocks a != b hold only
    Kt[a, b] times the velocity mass matrix;
  * space integrals use the 3-point Gauss rule per direction for r = 2 (exact
    for the convection integrand, of degree 3 r - 1 per direction) and the
    ceil(3 r / 2)-point rule for higher r.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import pressure_exponents
from .radau import dg_time_matrices

GAUSS3_S = np.array([0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)])
GAUSS3_W = np.array([5.0, 8.0, 5.0]) / 18.0


def _q2_1d(s):
    """Quadratic Lagrange basis at nodes 0, 1/2, 1 and derivatives, at points s."""
    s = np.asarray(s, dtype=np.float64)
    val = np.stack([(2 * s - 1) * (s - 1), 4 * s * (1 - s), s * (2 * s - 1)], axis=-1)
    der = np.stack([4 * s - 3, 4 - 8 * s, 4 * s - 1], axis=-1)
    return val, der


def _lagrange_1d(s, r):
    """Degree-r Lagrange basis at the equispaced nodes j / r of [0, 1] and derivatives, at s."""
    if r == 2:
        return _q2_1d(s)
    s = np.asarray(s, dtype=np.float64)
    t = np.arange(r + 1) / r
    val = np.ones(s.shape + (r + 1,))
    der = np.zeros(s.shape + (r + 1,))
    for j in range(r + 1):
        for m in range(r + 1):
            if m == j:
                continue
            f = (s - t[m]) / (t[j] - t[m])
            der[..., j] = der[..., j] * f + val[..., j] / (t[j] - t[m])
            val[..., j] = val[..., j] * f
    return val, der


def gauss_rule_01(r):
    """Gauss points and weights on [0, 1] for velocity degree r (3 points for r = 2)."""
    if r == 2:
        return GAUSS3_S, GAUSS3_W
    x, w = np.polynomial.legendre.leggauss((3 * r + 1) // 2)
    return 0.5 * (x + 1.0), 0.5 * w


def _tensor_points(point_sets):
    """Cartesian product of per-direction point sets, first direction fastest."""
    grids = np.meshgrid(*point_sets, indexing="ij")
    return np.stack([g.ravel(order="F") for g in grids], axis=1)


def tensor_basis(mesh, pts):
    """phi[q, n], dphi[q, n, i] (physical derivatives) for reference points pts[q, d]."""
    d = mesh.d
    off = mesh.local_node_offsets()
    vals, ders = [], []
    for i in range(d):
        v, dv = _lagrange_1d(pts[:, i], mesh.r)
        vals.append(v)
        ders.append(dv / mesh.h[i])
    nq, nl = pts.shape[0], mesh.n_loc_nodes
    phi = np.ones((nq, nl))
    for i in range(d):
        phi *= vals[i][:, off[:, i]]
    dphi = np.ones((nq, nl, d))
    for i in range(d):
        for j in range(d):
            dphi[:, :, i] *= (ders[j] if i == j else vals[j])[:, off[:, j]]
    return phi, dphi


def pressure_basis(pts, r=2):
    """P_{r-1}disc monomials in x^ = 2 s - 1 on [-1, 1]^d (numbering of `mesh.py`):
    {1, x^, y^(, z^)} for r = 2."""
    if r == 2:
        return np.concatenate([np.ones((pts.shape[0], 1)), 2 * pts - 1], axis=1)
    x = 2 * pts - 1
    return np.stack([np.prod(x ** np.array(e)[None, :], axis=1) for e in pressure_exponents(pts.shape[1], r)],
                    axis=1)


def volume_rule(mesh):
    gs, gw = gauss_rule_01(mesh.r)
    pts = _tensor_points([gs] * mesh.d)
    w = np.prod(_tensor_points([gw] * mesh.d), axis=1) * np.prod(mesh.h)
    return pts, w


def face_rule(mesh, axis, side):
    gs, gw = gauss_rule_01(mesh.r)
    sets = [gs] * mesh.d
    sets = list(sets)
    sets[axis] = np.array([float(side)])
    pts = _tensor_points(sets)
    wsets = [gw * mesh.h[j] if j != axis else np.array([1.0]) for j in range(mesh.d)]
    w = np.prod(_tensor_points(wsets), axis=1)
    return pts, w


def dirichlet_faces(mesh):
    """(axis, side) of Gamma_D: every boundary face except the outflow x = L_x."""
    return [(i, s) for i in range(mesh.d) for s in (0, 1) if not (i == 0 and s == 1)]


def boundary_cells(mesh, axis, side):
    ci = mesh.cell_index()
    target = 0 if side == 0 else mesh.shape[axis] - 1
    return np.nonzero(ci[:, axis] == target)[0]


def local_pattern(mesh):
    """Boolean [n_K, n_K] structural pattern of a cell's slab element matrix."""
    d, nl, nt = mesh.d, mesh.n_loc_nodes, mesh.n_time
    nv = d * nl
    ns = mesh.n_loc_space
    same = np.zeros((ns, ns), dtype=bool)
    same[:nv, :] = True
    same[nv:, :nv] = True
    cross = np.zeros((ns, ns), dtype=bool)
    cross[:nv, :nv] = np.kron(np.ones((nl, nl), dtype=bool), np.eye(d, dtype=bool))
    pat = np.zeros((mesh.n_K, mesh.n_K), dtype=bool)
    for a in range(nt):
        for b in range(nt):
            pat[a * ns:(a + 1) * ns, b * ns:(b + 1) * ns] = same if a == b else cross
    return pat


def element_matrices(mesh, V, nu, tau, gamma1=35.0, gamma2=35.0):
    """Dense slab element matrices E[cell, n_K, n_K] (row = test, col = trial).

    V[a, node, c] is the Newton linearisation state at Radau node a.
    """
    d, nl, nt, ns = mesh.d, mesh.n_loc_nodes, mesh.n_time, mesh.n_loc_space
    nv = d * nl
    nc = mesh.n_cells
    _, w_t, Kt, _ = dg_time_matrices(mesh.k)
    I_d = np.eye(d)

    pts, wq = volume_rule(mesh)
    phi, dphi = tensor_basis(mesh, pts)
    pib = pressure_basis(pts, mesh.r)
    npm = mesh.n_pmodes
    Mel = np.einsum("q,qn,qm->nm", wq, phi, phi)
    Sel = np.einsum("q,qni,qmi->nm", wq, dphi, dphi)
    Gel = -np.einsum("q,qp,qnc->ncp", wq, pib, dphi)       # [n, c, q]

    # Nitsche face matrices, one set per Dirichlet face orientation
    face_terms = []
    for axis, side in dirichlet_faces(mesh):
        fp, fw = face_rule(mesh, axis, side)
        fphi, fdphi = tensor_basis(mesh, fp)
        fpi = pressure_basis(fp, mesh.r)
        nrm = np.zeros(d)
        nrm[axis] = 2.0 * side - 1.0
        hF = mesh.h[axis]
        Fpen = np.einsum("q,qn,qm->nm", fw, fphi, fphi)
        Fdn = np.einsum("q,qn,qmi,i->nm", fw, fphi, fdphi, nrm)    # int (grad phi_m . n) phi_n
        vv = (np.kron(-nu * Fdn - nu * Fdn.T + gamma1 * nu / hF * Fpen, I_d)
              + gamma2 / hF * np.kron(Fpen, np.outer(nrm, nrm)))
        vp = np.einsum("q,qp,qn,c->ncp", fw, fpi, fphi, nrm).reshape(nv, npm)
        face_terms.append((boundary_cells(mesh, axis, side), vv, vp))

    cn = mesh.cell_nodes()
    E = np.zeros((nc, mesh.n_K, mesh.n_K))
    Mv = np.kron(Mel, I_d)
    Sv = np.kron(Sel, I_d)
    for a in range(nt):
        Vc = V[a][cn]                                    # [cell, n, c]
        vq = np.einsum("qn,knc->kqc", phi, Vc)
        gv = np.einsum("qni,knc->kqci", dphi, Vc)        # d_i v_c
        C1 = np.einsum("q,qn,kqi,qmi->knm", wq, phi, vq, dphi)
        C2 = np.einsum("q,qn,qm,kqce->kncme", wq, phi, phi, gv).reshape(nc, nv, nv)
        Aa = nu * Sv[None] + np.einsum("knm,ce->kncme", C1, I_d).reshape(nc, nv, nv) + C2
        Ga = np.broadcast_to(Gel.reshape(nv, npm), (nc, nv, npm)).copy()
        for cells, vv, vp in face_terms:
            Aa[cells] += vv
            Ga[cells] += vp
        s_a = slice(a * ns, a * ns + nv)
        p_a = slice(a * ns + nv, (a + 1) * ns)
        tw = tau * w_t[a]
        E[:, s_a, s_a] += tw * Aa
        E[:, s_a, p_a] += tw * Ga
        E[:, p_a, s_a] += tw * np.transpose(Ga, (0, 2, 1))
        for b in range(nt):
            s_b = slice(b * ns, b * ns + nv)
            E[:, s_a, s_b] += Kt[a, b] * Mv[None]
    return E


def assemble_jacobian(mesh, V, nu, tau, gamma1=35.0, gamma2=35.0):
    """Global slab Jacobian (scipy CSR, sorted columns, float64)."""
    E = element_matrices(mesh, V, nu, tau, gamma1, gamma2)
    pat = local_pattern(mesh)
    li, lj = np.nonzero(pat)
    dofs = mesh.cell_dofs().astype(np.int64)
    rows = dofs[:, li].ravel()
    cols = dofs[:, lj].ravel()
    vals = E[:, li, lj].ravel()
    del E
    J = sp.coo_matrix((vals, (rows, cols)), shape=(mesh.n, mesh.n)).tocsr()
    J.sum_duplicates()
    J.sort_indices()
    return J
