"""Time-marching workload: consecutive dG(k) slabs of a 2D channel with a
time-periodic inflow (the Newton iteration of Sec. 3 applied slab after slab,
Sec. 2 Eq. 2.2).

The slab problem F(X) = 0 and its Newton Jacobian come from `nonlinear.py` on
every level of a nested hierarchy; the coarse levels are rediscretised with the
Newton state injected at their Q2 nodes (as in `problems.py`).  The initial
velocity is the Poiseuille profile of the inflow peak at t = 0.

Inflow peak U(t) = 0.3 (1 + 0.5 sin(2 pi t / 0.5)): a period of 50 slabs at
tau = 0.01.
"""
from dataclasses import dataclass

import numpy as np

from .mesh import StructuredMesh, hierarchy_shapes
from .nonlinear import SlabOperator, extrapolation_matrix, inflow_amplitude, poiseuille_slab
from .problems import Level, H_CHANNEL
from .transfer import prolongation, inject_nodes

MARCH_CONFIGS = {
    # 200 slabs of 88 x 16 cells, dG(1), 4 levels (11 x 2 coarsest)
    "channel2d_88x16_k1_march": dict(shape=(88, 16), levels=4, k=1, nu=1e-3, tau=0.01, n_slabs=200),
}


@dataclass
class MarchLevelData:
    mesh: StructuredMesh
    op: SlabOperator
    P: object
    R: object
    inject: object    # fine node ids of this level's nodes on the next finer level (None on the finest)


class ChannelMarch:
    """Meshes, slab operators and transfers of the marching channel."""

    def __init__(self, shape=(88, 16), levels=4, k=1, nu=1e-3, tau=0.01, lengths=(2.2, H_CHANNEL),
                 inflow=(0.3, 0.5, 0.5)):
        """inflow = (U0, rel, period): peak U(t) = U0 (1 + rel sin(2 pi t / period))."""
        self.k, self.nu, self.tau = k, nu, tau
        self.inflow = tuple(inflow)
        shapes = hierarchy_shapes(shape, levels)
        meshes = [StructuredMesh(s, lengths, k) for s in shapes]
        self.levels = []
        for l, m in enumerate(meshes):
            if l > 0:
                P = prolongation(meshes[l - 1], m)
                R = P.T.tocsr()
                R.sort_indices()
            else:
                P = R = None
            inj = inject_nodes(m, meshes[l + 1]) if l + 1 < len(meshes) else None
            self.levels.append(MarchLevelData(mesh=m, op=SlabOperator(m, nu, tau), P=P, R=R, inject=inj))
        self.E = extrapolation_matrix(k)

    @property
    def fine(self):
        return self.levels[-1]

    @property
    def n(self):
        return self.fine.mesh.n

    def slab_start(self, n):
        """Start time of slab n (slabs are numbered from 1)."""
        return (n - 1) * self.tau

    def initial_slab(self):
        """Slab vector of the initial state on every time node (Poiseuille flow of U(0))."""
        return poiseuille_slab(self.fine.mesh, self.amplitude(0.0), self.nu)

    def amplitude(self, t):
        U0, rel, period = self.inflow
        return inflow_amplitude(t, U0, rel, period)

    def end_velocity(self, X):
        """Velocity at the slab's end point (its last Radau node, s = 1)."""
        m = self.fine.mesh
        return X.reshape(m.n_time, m.n_space)[-1, :m.n_vel].copy()

    def extrapolate(self, X_prev):
        """Fallback guess: the previous slab's time polynomial at the new Radau nodes."""
        m = self.fine.mesh
        return (self.E @ X_prev.reshape(m.n_time, m.n_space)).ravel()

    def residual(self, X, X_prev, n):
        """F(X) of slab n given the previous slab's solution."""
        return self.fine.op.residual(X, self.end_velocity(X_prev), self.slab_start(n), amplitude=self.amplitude)

    def hierarchy(self, X):
        """Newton Jacobians of the state X on every level, as `problems.Level` objects."""
        V = self.fine.op.velocity_state(X)
        states = [None] * len(self.levels)
        states[-1] = V
        for l in range(len(self.levels) - 2, -1, -1):
            states[l] = states[l + 1][:, self.levels[l].inject, :]
        out = []
        for l, L in enumerate(self.levels):
            m = L.mesh
            Xl = np.zeros(m.n)
            Xl.reshape(m.n_time, m.n_space)[:, :m.n_vel] = states[l].reshape(m.n_time, -1)
            out.append(Level(mesh=m, J=L.op.jacobian(Xl), P=L.P, R=L.R, cell_dofs=m.cell_dofs(),
                             colours=m.colours(), state=states[l]))
        return out

    def jacobian_values(self, X):
        """Only the CSR values of every level's Jacobian (the patterns never change)."""
        return [L.J.data for L in self.hierarchy(X)]
