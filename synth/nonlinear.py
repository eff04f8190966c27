"""Nonlinear dG(k) slab residual and its Newton Jacobian on one mesh, for time
marching (Sec. 2, Eq. 2.1 and 2.2; Sec. 3, Eq. 3.2 and 3.3; the Newton method of
Sec. 3 with the damping of the paper's solver description).

The discrete problem of slab n is F(X) = 0 with X the slab vector (time node
major, Eq. 3.2).  With the same readings as `assemble.py` (rows are test
functions; symmetric Nitsche on Gamma_D with gamma_1 = gamma_2 = 35; continuity
rows negated; (k+1)-point right Radau rule in time, so the spatial terms are
diagonal in time):

  F_a(X) = sum_b Kt[a,b] M u_b - c0[a] M u_prev
           + tau w_a [ nu S u_a + N(u_a) u_a + Nitsche(u_a) + G p_a - D g_a ]   (velocity rows)
  F_a(X) = tau w_a [ G^T u_a - Dp g_a ]                                          (pressure rows)

where N(u) is the convection form ((u . grad) dv, psi), g_a the Dirichlet data at
time node a (the inflow profile at x = 0, zero on the walls) and D, Dp the data
parts of the Nitsche terms.  The Newton Jacobian adds ((dv . grad) u, psi) to
N(u); it equals `assemble_jacobian` for the same state (tested).

Everything that does not depend on the state is computed once per mesh, and the
CSR pattern is fixed, so repeated Jacobians reuse one scatter map.
"""
import numpy as np
import scipy.sparse as sp

from .assemble import (volume_rule, tensor_basis, pressure_basis, face_rule, dirichlet_faces,
                       boundary_cells, local_pattern)
from .radau import dg_time_matrices, lagrange_at_nodes


def poiseuille(y, H, U):
    """Parabolic channel profile of peak U on [0, H]."""
    return 4.0 * U * y * (H - y) / H ** 2


def inflow_amplitude(t, U0=0.3, rel=0.5, period=0.5):
    """Time-periodic inflow peak U(t) = U0 (1 + rel sin(2 pi t / period))."""
    return U0 * (1.0 + rel * np.sin(2.0 * np.pi * t / period))


class SlabOperator:
    """F(X), J(X) of one slab on one mesh (2D or 3D channel, inflow at x = 0)."""

    def __init__(self, mesh, nu, tau, gamma1=35.0, gamma2=35.0):
        if mesh.r != 2:
            raise NotImplementedError("the slab operator is written for Q2 x P1disc (r = 2)")
        self.mesh, self.nu, self.tau = mesh, float(nu), float(tau)
        d, nl, nt, ns = mesh.d, mesh.n_loc_nodes, mesh.n_time, mesh.n_loc_space
        nv = d * nl
        nc = mesh.n_cells
        self.s, self.w, self.Kt, self.c0 = dg_time_matrices(mesh.k)
        I_d = np.eye(d)
        pts, wq = volume_rule(mesh)
        phi, dphi = tensor_basis(mesh, pts)
        pib = pressure_basis(pts)
        self.phi, self.dphi, self.wq = phi, dphi, wq
        Mel = np.einsum("q,qn,qm->nm", wq, phi, phi)
        Sel = np.einsum("q,qni,qmi->nm", wq, dphi, dphi)
        Gel = -np.einsum("q,qp,qnc->ncp", wq, pib, dphi).reshape(nv, d + 1)
        self.Mv = np.kron(Mel, I_d)
        # state-independent spatial blocks per cell: viscosity + Nitsche, and the pressure coupling
        A0 = np.broadcast_to(nu * np.kron(Sel, I_d), (nc, nv, nv)).copy()
        G = np.broadcast_to(Gel, (nc, nv, d + 1)).copy()
        # data of a unit inflow profile (peak 1) on the inflow face
        gdat = np.zeros((nc, nv + d + 1))
        xyz = mesh.node_coords()
        cn = mesh.cell_nodes()
        prof = np.ones(mesh.n_nodes)
        for i, h in enumerate(mesh.lengths[1:]):
            prof *= poiseuille(xyz[:, 1 + i], h, 1.0)
        for axis, side in dirichlet_faces(mesh):
            fp, fw = face_rule(mesh, axis, side)
            fphi, fdphi = tensor_basis(mesh, fp)
            fpi = pressure_basis(fp)
            nrm = np.zeros(d)
            nrm[axis] = 2.0 * side - 1.0
            hF = mesh.h[axis]
            Fpen = np.einsum("q,qn,qm->nm", fw, fphi, fphi)
            Fdn = np.einsum("q,qn,qmi,i->nm", fw, fphi, fdphi, nrm)
            vv = (np.kron(-nu * Fdn - nu * Fdn.T + gamma1 * nu / hF * Fpen, I_d)
                  + gamma2 / hF * np.kron(Fpen, np.outer(nrm, nrm)))
            vp = np.einsum("q,qp,qn,c->ncp", fw, fpi, fphi, nrm).reshape(nv, d + 1)
            cells = boundary_cells(mesh, axis, side)
            A0[cells] += vv
            G[cells] += vp
            if axis == 0 and side == 0:
                # data parts: the symmetry and penalty terms act on (u - g), the pressure row on (u - g) . n
                Dv = (np.kron(-nu * Fdn.T + gamma1 * nu / hF * Fpen, I_d)
                      + gamma2 / hF * np.kron(Fpen, np.outer(nrm, nrm)))
                gl = np.zeros((len(cells), nl, d))
                gl[:, :, 0] = prof[cn[cells]]
                gl = gl.reshape(len(cells), nv)
                gdat[cells, :nv] += gl @ Dv.T
                gdat[cells, nv:] += gl @ vp
        self.A0, self.G = A0, G
        # global unit-data vector of one time node (spatial numbering)
        sdofs = mesh.cell_dofs_space()
        self.g_unit = np.bincount(sdofs.ravel(), weights=gdat.ravel(), minlength=mesh.n_space)
        self.cn = cn
        self.dofs = mesh.cell_dofs().astype(np.int64)
        # global velocity mass (spatial velocity numbering)
        vd = sdofs[:, :nv]
        li, lj = np.meshgrid(np.arange(nv), np.arange(nv), indexing="ij")
        self.Mglob = sp.coo_matrix((np.broadcast_to(self.Mv, (nc, nv, nv)).ravel(),
                                    (vd[:, li].ravel(), vd[:, lj].ravel())),
                                   shape=(mesh.n_vel, mesh.n_vel)).tocsr()
        # fixed CSR pattern and the scatter map of the element entries into it
        pat = local_pattern(mesh)
        self.li, self.lj = np.nonzero(pat)
        rows = self.dofs[:, self.li].ravel()
        cols = self.dofs[:, self.lj].ravel()
        keys = rows * mesh.n + cols
        uk, inv = np.unique(keys, return_inverse=True)
        self.scatter = inv
        self.nnz = len(uk)
        urow = uk // mesh.n
        self.indices = (uk % mesh.n).astype(np.int32)
        self.indptr = np.concatenate([[0], np.cumsum(np.bincount(urow, minlength=mesh.n))]).astype(np.int64)
        # quadrature products for the convection terms
        self.Wphi = wq[:, None] * phi                                  # [q, n]
        self.PP = (wq[:, None, None] * phi[:, :, None] * phi[:, None, :]).reshape(len(wq), nl * nl)

    # ---- element blocks ------------------------------------------------------------
    def _convection(self, Va, newton):
        """Per-cell velocity blocks [nc, nv, nv] of N(V) (and of the Newton term)."""
        m = self.mesh
        d, nl, nc = m.d, m.n_loc_nodes, m.n_cells
        Vc = Va[self.cn]                                               # [cell, n, c]
        vq = np.einsum("qn,knc->kqc", self.phi, Vc)                    # [cell, q, c]
        T = np.einsum("kqi,qmi->kqm", vq, self.dphi)                   # (v . grad) phi_m at q
        C1 = np.einsum("qn,kqm->knm", self.Wphi, T)
        out = np.einsum("knm,ce->kncme", C1, np.eye(d)).reshape(nc, d * nl, d * nl)
        if newton:
            gv = np.einsum("qni,knc->kqci", self.dphi, Vc).reshape(nc, len(self.wq), d * d)
            C2 = np.einsum("kqx,qy->kxy", gv, self.PP).reshape(nc, d, d, nl, nl)
            out += C2.transpose(0, 3, 1, 4, 2).reshape(nc, d * nl, d * nl)
        return out

    def element_matrices(self, V, newton=True):
        """Slab element matrices [nc, n_K, n_K]; V[a, node, c] the velocity state."""
        m = self.mesh
        d, nl, nt, ns = m.d, m.n_loc_nodes, m.n_time, m.n_loc_space
        nv = d * nl
        E = np.zeros((m.n_cells, m.n_K, m.n_K))
        for a in range(nt):
            Aa = self.A0 + self._convection(V[a], newton)
            s_a = slice(a * ns, a * ns + nv)
            p_a = slice(a * ns + nv, (a + 1) * ns)
            tw = self.tau * self.w[a]
            E[:, s_a, s_a] += tw * Aa
            E[:, s_a, p_a] += tw * self.G
            E[:, p_a, s_a] += tw * np.transpose(self.G, (0, 2, 1))
            for b in range(nt):
                E[:, s_a, b * ns:b * ns + nv] += self.Kt[a, b] * self.Mv[None]
        return E

    # ---- global operators ----------------------------------------------------------
    def velocity_state(self, X):
        """V[a, node, c] from a slab vector."""
        m = self.mesh
        return X.reshape(m.n_time, m.n_space)[:, :m.n_vel].reshape(m.n_time, m.n_nodes, m.d)

    def jacobian(self, X):
        """Newton Jacobian J(X) (CSR, sorted columns, the same pattern for every X)."""
        E = self.element_matrices(self.velocity_state(X), newton=True)
        vals = E[:, self.li, self.lj].ravel()
        data = np.bincount(self.scatter, weights=vals, minlength=self.nnz)
        return sp.csr_matrix((data, self.indices.copy(), self.indptr.copy()), shape=(self.mesh.n, self.mesh.n))

    def residual(self, X, u_prev, t0, amplitude=inflow_amplitude):
        """F(X) of the slab [t0, t0 + tau] with previous end velocity u_prev (n_vel) and
        inflow peak amplitude(t)."""
        m = self.mesh
        E = self.element_matrices(self.velocity_state(X), newton=False)
        loc = np.einsum("kij,kj->ki", E, X[self.dofs])
        F = np.bincount(self.dofs.ravel(), weights=loc.ravel(), minlength=m.n)
        F = F.reshape(m.n_time, m.n_space)
        Mu = self.Mglob @ u_prev
        for a in range(m.n_time):
            F[a, :m.n_vel] -= self.c0[a] * Mu
            F[a] -= self.tau * self.w[a] * amplitude(t0 + self.tau * self.s[a]) * self.g_unit
        return F.ravel()


def extrapolation_matrix(k):
    """E[a, b] = chi_b(1 + s_a): the previous slab's Lagrange time polynomial
    evaluated at the next slab's Radau nodes."""
    s, _, _, _ = dg_time_matrices(k)
    chi = lagrange_at_nodes(s)
    from numpy.polynomial import polynomial as nppoly
    return np.array([[nppoly.polyval(1.0 + s[a], chi[b]) for b in range(k + 1)] for a in range(k + 1)])


def poiseuille_slab(mesh, U, nu):
    """Slab vector of steady Poiseuille flow (peak U, do-nothing outflow p = 0 at
    x = L_x) on every time node: the exact solution of the 2D channel for a constant
    inflow (Q2 velocities and P1disc pressures represent it exactly)."""
    if mesh.d != 2:
        raise ValueError("the closed form is the 2D channel's")
    H = mesh.lengths[1]
    L = mesh.lengths[0]
    xyz = mesh.node_coords()
    sp_vec = np.zeros(mesh.n_space)
    u = np.ones(mesh.n_nodes) * U
    for i, h in enumerate(mesh.lengths[1:]):
        u *= poiseuille(xyz[:, 1 + i], h, 1.0)
    sp_vec[0:mesh.n_vel:mesh.d] = u
    # p = 8 nu U / H^2 (L - x); P1disc coefficients {1, x^, y^} per cell
    ci = mesh.cell_index()
    xc = (ci[:, 0] + 0.5) * mesh.h[0]
    g = 8.0 * nu * U / H ** 2
    pc = np.zeros((mesh.n_cells, 3))
    pc[:, 0] = g * (L - xc)
    pc[:, 1] = -g * mesh.h[0] / 2.0
    sp_vec[mesh.n_vel:] = pc.ravel()
    return np.tile(sp_vec, mesh.n_time)
