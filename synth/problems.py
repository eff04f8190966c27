"""Seeded synthetic workloads.

The paper's benchmark (flow around a cylinder, Sec. 4) needs geometry that is
not available here; the workloads are cylinder-free channels/boxes of the same
outer extents with Newton linearisation states and right-hand sides drawn from
fixed seeds.  The state on the finest level is a parabolic inflow profile of
peak U in x-direction plus i.i.d. uniform noise of 5 % of U on every velocity
DoF and Radau node; coarse levels take the injected fine state (their Q2 nodes
are fine Q2 nodes).  Every level is rediscretised with its own h.
The right-hand side is i.i.d. N(0, 1) on the finest level.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .mesh import StructuredMesh, hierarchy_shapes
from .assemble import assemble_jacobian
from .assemble_chunked import assemble_jacobian_chunked

# element-matrix entries above which a level is assembled chunk by chunk straight into CSR
CHUNKED_ASSEMBLY_ENTRIES = 2e7
from .transfer import prolongation, inject_nodes

H_CHANNEL = 0.41

# name -> parameters; the finest shape, number of levels and k define the sizes
CONFIGS = {
    "channel2d_44x8_k1": dict(d=2, shape=(44, 8), lengths=(2.2, H_CHANNEL), levels=3, k=1,
                              nu=1e-3, tau=0.01, U=0.3, seed=0),
    "channel2d_176x32_k2": dict(d=2, shape=(176, 32), lengths=(2.2, H_CHANNEL), levels=5, k=2,
                                nu=1e-3, tau=0.01, U=0.3, seed=1),
    "box3d_100x16x16_k1": dict(d=3, shape=(100, 16, 16), lengths=(2.5, H_CHANNEL, H_CHANNEL),
                               levels=4, k=1, nu=1e-3, tau=0.01, U=0.45, seed=2),
    "channel2d_88x16_k1": dict(d=2, shape=(88, 16), lengths=(2.2, H_CHANNEL), levels=4, k=1,
                               nu=1e-3, tau=0.01, U=0.3, seed=4),
}


@dataclass
class Level:
    mesh: StructuredMesh
    J: sp.csr_matrix
    P: Optional[sp.csr_matrix]       # level l-1 -> l (None on level 0)
    R: Optional[sp.csr_matrix]       # = P^T as its own CSR
    cell_dofs: np.ndarray             # int32 [n_cells, n_K]
    colours: np.ndarray               # int32 [n_cells]
    state: np.ndarray                 # [n_time, n_nodes, d] linearisation state

    @property
    def n(self):
        return self.mesh.n

    def colour_order(self):
        """(cells sorted by colour, ascending inside a colour; colour offsets)."""
        order = np.argsort(self.colours, kind="stable").astype(np.int32)
        counts = np.bincount(self.colours, minlength=self.mesh.n_colours)
        ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        return order, ptr


@dataclass
class Problem:
    name: str
    params: dict
    levels: List[Level] = field(default_factory=list)   # 0 = coarsest
    b: Optional[np.ndarray] = None

    @property
    def finest(self):
        return self.levels[-1]


def inflow_state(mesh, U, rng, noise=0.05):
    """Parabolic profile of peak U in x plus uniform noise of `noise` * U."""
    xyz = mesh.node_coords()
    H = mesh.lengths[1:]
    prof = np.ones(mesh.n_nodes)
    for i, h in enumerate(H):
        y = xyz[:, 1 + i]
        prof *= 4.0 * y * (h - y) / h ** 2
    V = np.zeros((mesh.n_time, mesh.n_nodes, mesh.d))
    V[:, :, 0] = U * prof
    V += rng.uniform(-noise * U, noise * U, size=V.shape)
    return V


def build_hierarchy(d, shape, lengths, levels, k, nu, tau, U, seed=0, noise=0.05, state=None, shapes=None, r=2):
    """Levels 0 (coarsest) .. levels-1 of one problem (velocity degree r); `shapes` overrides the
    coarsening rule."""
    if shapes is None:
        shapes = hierarchy_shapes(shape, levels)
    levels = len(shapes)
    meshes = [StructuredMesh(s, lengths, k, r) for s in shapes]
    fine = meshes[-1]
    if state is None:
        state = inflow_state(fine, U, np.random.default_rng(1000 + seed), noise)
    states = [None] * levels
    states[-1] = state
    for l in range(levels - 2, -1, -1):
        states[l] = states[l + 1][:, inject_nodes(meshes[l], meshes[l + 1]), :]
    out = []
    for l, m in enumerate(meshes):
        if m.r == 2 and m.n_cells * m.n_K ** 2 > CHUNKED_ASSEMBLY_ENTRIES:
            J = assemble_jacobian_chunked(m, states[l], nu, tau)
        else:
            J = assemble_jacobian(m, states[l], nu, tau)
        if l > 0:
            P = prolongation(meshes[l - 1], m)
            R = P.T.tocsr()
            R.sort_indices()
        else:
            P = R = None
        out.append(Level(mesh=m, J=J, P=P, R=R, cell_dofs=m.cell_dofs(), colours=m.colours(),
                         state=states[l]))
    return out


def build_problem(name=None, **overrides):
    """Build a named workload (see CONFIGS) or a custom one from keyword args."""
    params = dict(CONFIGS[name]) if name is not None else {}
    params.update(overrides)
    p = dict(params)
    seed = p.pop("seed", 0)
    noise = p.pop("noise", 0.05)
    p.pop("d", None)
    d = len(p["shape"])
    levels = build_hierarchy(d=d, seed=seed, noise=noise, **p)
    b = np.random.default_rng(2000 + seed).standard_normal(levels[-1].n)
    return Problem(name=name or "custom", params=params, levels=levels, b=b)
