"""Structured quadrilateral/hexahedral meshes with Q_r x P_{r-1}disc degrees of freedom.

Sec. 2: each multigrid level T_l is a decomposition of the domain into quads
(d = 2) or hexahedra (d = 3); velocities are continuous (Q_r)^d and pressures
discontinuous P_{r-1}: r = 2 by default, r = 4 in the paper's 2D study.  The
meshes are uniform boxes, refined by two in every direction that is halved
(h_l = h_{l-1}/2 there).

Numbering (one time node; Eq. 3.2 orders the slab vector node by node in time):
  * Q_r nodes form a (r n_0 + 1) x ... grid, first index fastest.
  * velocity DoF = node * d + component (components interleaved),
  * pressure DoF = d * n_nodes + cell * m + q with m = C(r - 1 + d, d) monomials
    of total degree <= r - 1 in the reference coordinates of [-1, 1]^d, by degree
    and, within a degree, by decreasing exponent of x^ first: {1, x^, y^(, z^)}
    for r = 2,
  * slab DoF = a * n_space + spatial DoF, a = 0..k the Radau node.
The patch of a cell K (the local numbering dof(K, mu^) of Sec. 3) lists, for
each time node a in turn, the (r + 1)^d local nodes (first index fastest) with
interleaved components, then the m pressure coefficients, so that
n_K = (k + 1) ((r + 1)^d d + m): for r = 2, 42 / 63 / 84 in 2D (k = 1, 2, 3) and
170 in 3D (k = 1); for r = 4 in 2D, 60 (k + 1).
"""
from math import comb

import numpy as np


def pressure_exponents(d, r):
    """Exponent tuples of the P_{r-1} monomials, in the pressure numbering order."""
    out = []
    for deg in range(r):
        def rec(prefix, left, dims):
            if dims == 1:
                out.append(tuple(prefix + [left]))
                return
            for e in range(left, -1, -1):
                rec(prefix + [e], left - e, dims - 1)
        rec([], deg, d)
    return out


def coarsen_shape(shape):
    """Halve every direction whose cell count is even and at least 4."""
    return tuple(n // 2 if (n % 2 == 0 and n >= 4) else n for n in shape)


def hierarchy_shapes(fine_shape, n_levels):
    """Cell counts of levels 0 (coarsest) .. n_levels-1 (finest)."""
    shapes = [tuple(fine_shape)]
    for _ in range(n_levels - 1):
        c = coarsen_shape(shapes[0])
        if c == shapes[0]:
            raise ValueError(f"mesh {fine_shape} cannot be coarsened {n_levels - 1} times")
        shapes.insert(0, c)
    return shapes


class StructuredMesh:
    def __init__(self, shape, lengths, k, r=2):
        self.d = len(shape)
        if self.d not in (2, 3):
            raise ValueError("d must be 2 or 3")
        self.r = int(r)
        if self.r < 2:
            raise ValueError("velocity degree r must be at least 2")
        self.shape = tuple(int(n) for n in shape)
        self.lengths = tuple(float(L) for L in lengths)
        self.h = tuple(L / n for L, n in zip(self.lengths, self.shape))
        self.k = int(k)
        self.node_shape = tuple(self.r * n + 1 for n in self.shape)
        self.n_nodes = int(np.prod(self.node_shape))
        self.n_cells = int(np.prod(self.shape))
        self.n_loc_nodes = (self.r + 1) ** self.d
        self.n_pmodes = comb(self.r - 1 + self.d, self.d)
        self.n_vel = self.d * self.n_nodes
        self.n_pres = self.n_pmodes * self.n_cells
        self.n_space = self.n_vel + self.n_pres
        self.n_time = self.k + 1
        self.n = self.n_time * self.n_space
        self.n_loc_space = self.d * self.n_loc_nodes + self.n_pmodes
        self.n_K = self.n_time * self.n_loc_space

    # ---- indices -------------------------------------------------------
    def cell_index(self):
        """[n_cells, d] integer cell coordinates (first index fastest)."""
        idx = np.unravel_index(np.arange(self.n_cells), self.shape, order="F")
        return np.stack(idx, axis=1)

    def node_index(self):
        idx = np.unravel_index(np.arange(self.n_nodes), self.node_shape, order="F")
        return np.stack(idx, axis=1)

    def node_coords(self):
        return self.node_index() * (np.array(self.h) / float(self.r))

    def local_node_offsets(self):
        """[(r + 1)^d, d] offsets (0 .. r) of the local nodes, first index fastest."""
        idx = np.unravel_index(np.arange(self.n_loc_nodes), (self.r + 1,) * self.d, order="F")
        return np.stack(idx, axis=1)

    def cell_nodes(self):
        """[n_cells, (r + 1)^d] global node ids of each cell."""
        ci = self.cell_index()
        off = self.local_node_offsets()
        g = self.r * ci[:, None, :] + off[None, :, :]
        strides = np.cumprod((1,) + self.node_shape[:-1])
        return (g * strides).sum(axis=2)

    def cell_dofs_space(self):
        """[n_cells, n_loc_space] spatial DoFs of each cell (velocity, then pressure)."""
        cn = self.cell_nodes()
        d = self.d
        vel = (cn[:, :, None] * d + np.arange(d)[None, None, :]).reshape(self.n_cells, -1)
        m = self.n_pmodes
        pres = self.n_vel + np.arange(self.n_cells)[:, None] * m + np.arange(m)[None, :]
        return np.concatenate([vel, pres], axis=1)

    def cell_dofs(self):
        """[n_cells, n_K] int32 slab DoFs of each cell, time node by time node."""
        sp = self.cell_dofs_space()
        blocks = [sp + a * self.n_space for a in range(self.n_time)]
        return np.concatenate(blocks, axis=1).astype(np.int32)

    def colours(self):
        """Cell colour sum_i (c_i mod 2) 2^i: same-colour cells share no node."""
        ci = self.cell_index()
        return ((ci % 2) * (1 << np.arange(self.d))[None, :]).sum(axis=1).astype(np.int32)

    @property
    def n_colours(self):
        return 1 << self.d
