"""Slab Jacobian assembly for large meshes, cell chunk by cell chunk, straight
into CSR (the same operator as `assemble.py`: Sec. 2, Eq. 2.1 and 2.2; Sec. 3,
Eq. 3.2 and 3.3, with the readings listed there).

`assemble_jacobian` builds one dense element matrix per cell and sums a COO
list, which needs tens of GB for the 3D box.  Here the CSR structure is known
in closed form on the structured mesh, so every element entry goes to its
position in the CSR arrays directly:

  * the velocity row of Q2 node g (component c, Radau node a) holds, for every
    Radau node b, the nodes of the box B(g) spanned by the cells that contain
    g (in 1D: g -2 .. g +2 at a cell vertex, g -1 .. g +1 inside a cell,
    clipped to the mesh), all d components when b = a and component c
    otherwise, and for b = a the P1disc coefficients of the cells containing
    g; columns ascend (time node, then spatial DoF: nodes in increasing id,
    components interleaved, pressures after all velocities);
  * the pressure row of cell K (coefficient q, node a) holds the velocities of
    K's 3^d nodes at node a.

Cells of one colour share no DoF, so within a colour each CSR position
receives at most one contribution per chunk and the sums need no sorting.  The
result equals `assemble_jacobian` (same pattern, values up to the order of the
floating-point sums; tested on small meshes).
"""
import numpy as np
import scipy.sparse as sp

from .assemble import (volume_rule, tensor_basis, pressure_basis, face_rule, dirichlet_faces,
                       boundary_cells, local_pattern)
from .radau import dg_time_matrices


class ChunkedJacobian:
    def __init__(self, mesh, nu, tau, gamma1=35.0, gamma2=35.0, chunk=512, threads=8):
        if mesh.r != 2:
            raise NotImplementedError("the chunked assembler is written for Q2 x P1disc (r = 2)")
        self.mesh, self.nu, self.tau, self.chunk = mesh, float(nu), float(tau), int(chunk)
        self.threads = int(threads)
        d, nl = mesh.d, mesh.n_loc_nodes
        nv = d * nl
        I_d = np.eye(d)
        _, self.w, self.Kt, _ = dg_time_matrices(mesh.k)
        pts, wq = volume_rule(mesh)
        phi, dphi = tensor_basis(mesh, pts)
        pib = pressure_basis(pts)
        self.phi, self.dphi, self.wq = phi, dphi, wq
        Mel = np.einsum("q,qn,qm->nm", wq, phi, phi)
        Sel = np.einsum("q,qni,qmi->nm", wq, dphi, dphi)
        self.Mv = np.kron(Mel, I_d)
        self.A_in = nu * np.kron(Sel, I_d)
        self.G_in = -np.einsum("q,qp,qnc->ncp", wq, pib, dphi).reshape(nv, d + 1)
        self.Wphi = wq[:, None] * phi
        self.PP = (wq[:, None, None] * phi[:, :, None] * phi[:, None, :]).reshape(len(wq), nl * nl)
        # Nitsche face terms and, per cell, which faces it carries
        self.faces = []
        on_face = np.zeros((mesh.n_cells, 2 * d), dtype=bool)
        for f, (axis, side) in enumerate(dirichlet_faces(mesh)):
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
            self.faces.append((vv, vp))
            on_face[boundary_cells(mesh, axis, side), f] = True
        self.on_face = on_face[:, :len(self.faces)]
        self.cn = mesh.cell_nodes()
        self.ci = mesh.cell_index()
        self.cds = mesh.cell_dofs_space().astype(np.int64)
        self.li, self.lj = np.nonzero(local_pattern(mesh))
        self._pattern()

    # ---- CSR structure -----------------------------------------------------------------------
    def _node_boxes(self):
        """Per node: lower corner and extents of the node box B(g) and of the cell box."""
        m = self.mesh
        g = m.node_index()
        lo = np.empty_like(g)
        ext = np.empty_like(g)
        clo = np.empty_like(g)
        cext = np.empty_like(g)
        for i in range(m.d):
            gi, N = g[:, i], m.shape[i]
            even = gi % 2 == 0
            c_lo = np.where(even, np.maximum(gi // 2 - 1, 0), (gi - 1) // 2)
            c_hi = np.where(even, np.minimum(gi // 2, N - 1), (gi - 1) // 2)
            clo[:, i], cext[:, i] = c_lo, c_hi - c_lo + 1
            lo[:, i], ext[:, i] = 2 * c_lo, 2 * (c_hi - c_lo + 1) + 1
        return lo, ext, clo, cext

    def _pattern(self):
        m = self.mesh
        d, nt = m.d, m.n_time
        self.lo, self.ext, self.clo, self.cext = self._node_boxes()
        B = np.prod(self.ext, axis=1)
        C = np.prod(self.cext, axis=1)
        self.B, self.C = B, C
        vel_len = B * (d + nt - 1) + C * (d + 1)                     # per node
        space_len = np.concatenate([np.repeat(vel_len, d), np.full(m.n_pres, (3 ** d) * d)])
        lens = np.tile(space_len, nt)
        self.indptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        self.nnz = int(self.indptr[-1])

    def _cell_class(self, cells):
        """Per cell and direction: whether a neighbour cell exists below / above.  Ranks of
        the element entries inside their rows depend on the cell only through this."""
        m = self.mesh
        ci = self.ci[cells]
        cls = np.zeros(len(cells), dtype=np.int64)
        for i in range(m.d):
            code = (ci[:, i] > 0).astype(np.int64) + 2 * (ci[:, i] < m.shape[i] - 1)
            cls = cls * 4 + code
        return cls

    def _positions(self, cells):
        """CSR positions and column ids of the local pattern entries of `cells`."""
        m = self.mesh
        d, nl = m.d, m.n_loc_nodes
        nv, ns = d * nl, m.n_loc_space
        li, lj = self.li, self.lj
        ta, sa = li // ns, li % ns                                     # row: time node, local spatial
        tb, sb = lj // ns, lj % ns
        cds = self.cds[cells]                                          # [c, ns] spatial DoFs
        cols = (tb * m.n_space)[None, :] + cds[:, sb]
        rows = (ta * m.n_space)[None, :] + cds[:, sa]
        if not hasattr(self, "_rank_table"):
            self._rank_table = {}
        cls = self._cell_class(cells)
        rank = np.empty(rows.shape, dtype=np.int64)
        for c in np.unique(cls):
            sel = cls == c
            if c not in self._rank_table:
                self._rank_table[c] = self._rank(cells[sel][:1])[0]
            rank[sel] = self._rank_table[c][None, :]
        return self.indptr[rows] + rank, cols

    def _rank(self, cells):
        """Rank of every local pattern entry's column inside its CSR row (closed form)."""
        m = self.mesh
        d, nl = m.d, m.n_loc_nodes
        nv, ns = d * nl, m.n_loc_space
        li, lj = self.li, self.lj
        ta, sa = li // ns, li % ns
        tb, sb = lj // ns, lj % ns
        cn = self.cn[cells]
        vel_row = sa < nv
        g = cn[:, np.minimum(sa, nv - 1) // d]                         # row node (velocity rows)
        lo, ext, clo, cext = self.lo[g], self.ext[g], self.clo[g], self.cext[g]
        Bg, Cg = self.B[g], self.C[g]
        blk_a = Bg * d + Cg * (d + 1)
        b_, a_ = tb[None, :], ta[None, :]
        prefix = b_ * Bg + np.where(b_ > a_, blk_a - Bg, 0)
        gcol = cn[:, np.minimum(sb, nv - 1) // d]                      # column node (velocity columns)
        gidx = m.node_index()[gcol] - lo                               # [c, e, d]
        didx = np.zeros_like(Bg)
        cell_idx = np.zeros_like(Bg)
        cc = self.ci[cells][:, None, :] - clo                          # [c, e, d]
        stride = np.ones_like(Bg)
        cstride = np.ones_like(Bg)
        for i in range(d):
            didx += gidx[:, :, i] * stride
            stride *= ext[:, :, i]
            cell_idx += cc[:, :, i] * cstride
            cstride *= cext[:, :, i]
        vel_col = (sb < nv)[None, :]
        rank_vv = prefix + np.where(b_ == a_, d * didx + (sb % d)[None, :], didx)
        rank_vp = prefix + Bg * d + cell_idx * (d + 1) + (sb - nv)[None, :]
        rank_v = np.where(vel_col, rank_vv, rank_vp)
        # pressure rows: velocities of the cell's nodes at the same time node
        rank_p = d * (np.minimum(sb, nv - 1) // d) + (sb % d)
        return np.where(vel_row[None, :], rank_v, rank_p[None, :])

    # ---- element blocks -----------------------------------------------------------------------
    def _elements(self, cells, V):
        m = self.mesh
        d, nl, nt, ns = m.d, m.n_loc_nodes, m.n_time, m.n_loc_space
        nv = d * nl
        nc = len(cells)
        A0 = np.broadcast_to(self.A_in, (nc, nv, nv)).copy()
        G = np.broadcast_to(self.G_in, (nc, nv, d + 1)).copy()
        onf = self.on_face[cells]
        for f, (vv, vp) in enumerate(self.faces):
            sel = onf[:, f]
            A0[sel] += vv
            G[sel] += vp
        E = np.zeros((nc, m.n_K, m.n_K))
        cn = self.cn[cells]
        nq = len(self.wq)
        for a in range(nt):
            Vc = V[a][cn]                                              # [c, n, comp]
            vq = np.matmul(self.phi[None], Vc)                         # [c, q, comp]
            # (v . grad) phi_m at q, then C1[k, n, m] = sum_q w phi_n (v . grad phi_m)
            T = np.einsum("kqi,qmi->kqm", vq, self.dphi, optimize=True)
            C1 = np.matmul(self.Wphi.T[None], T)                       # [c, n, m]
            conv = np.zeros((nc, nl, d, nl, d))
            for c in range(d):
                conv[:, :, c, :, c] = C1
            conv = conv.reshape(nc, nv, nv)
            # grad v at q: gv[k, q, c, i] = sum_n dphi[q, n, i] V[k, n, c]
            gv = np.einsum("qni,knc->kqci", self.dphi, Vc, optimize=True).reshape(nc, nq, d * d)
            C2 = np.matmul(gv.transpose(0, 2, 1), self.PP).reshape(nc, d, d, nl, nl)
            conv += C2.transpose(0, 3, 1, 4, 2).reshape(nc, nv, nv)
            tw = self.tau * self.w[a]
            s_a = slice(a * ns, a * ns + nv)
            p_a = slice(a * ns + nv, (a + 1) * ns)
            E[:, s_a, s_a] = tw * (A0 + conv)
            E[:, s_a, p_a] = tw * G
            E[:, p_a, s_a] = tw * np.transpose(G, (0, 2, 1))
            for b in range(nt):
                E[:, s_a, b * ns:b * ns + nv] += self.Kt[a, b] * self.Mv[None]
        return E[:, self.li, self.lj]

    def jacobian(self, V):
        """CSR (int64 row pointers, int32 sorted columns) of the Newton Jacobian at state V."""
        m = self.mesh
        data = np.zeros(self.nnz)
        indices = np.full(self.nnz, -1, dtype=np.int64)
        col = m.colours()
        self._positions(np.arange(min(m.n_cells, 1)))  # rank tables are filled by one thread

        def work(cells):
            pos, cols = self._positions(cells)
            vals = self._elements(cells, V)
            data[pos] += vals          # chunks of one colour touch disjoint positions
            indices[pos] = cols

        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=self.threads) as ex:
            for c in range(m.n_colours):
                cells_c = np.nonzero(col == c)[0]
                list(ex.map(work, [cells_c[s:s + self.chunk] for s in range(0, len(cells_c), self.chunk)]))
        if (indices < 0).any():
            raise AssertionError("pattern position not covered by any element")
        J = sp.csr_matrix((data, indices.astype(np.int32), self.indptr), shape=(m.n, m.n))
        J.has_sorted_indices = True
        return J


def assemble_jacobian_chunked(mesh, V, nu, tau, chunk=512):
    return ChunkedJacobian(mesh, nu, tau, chunk=chunk).jacobian(V)
