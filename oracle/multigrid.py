"""Geometric-multigrid V-cycle, FP64 oracle (Sec. 3).

On the coarsest partition T_0 the defect equation J_0 d_0 = b_0 is solved by a
direct solver (here dense LU with partial pivoting, LAPACK getrf/getrs through
SciPy).  On T_l, l >= 1, the V-cycle smooths nu_1 times from d = 0 with the
Vanka iteration, restricts the defect b - J_l d with R_l, recurses, adds the
prolonged coarse correction P_l e and smooths nu_2 times.
"""
import numpy as np
import scipy.linalg as sla

from .vanka import setup_level, smooth


class OracleHierarchy:
    """Holds J_l, P_l, R_l, cell maps and the setup results of every level.

    levels: sequence of objects or dicts with J, P, R, cell_dofs, colours
    (index 0 = coarsest).  `patch_store` optionally maps the FP64 inverses to
    the values actually applied (FP32 / BF16 rounding).
    """

    def __init__(self, levels, omega=0.7, mode="additive", order="coloured", patch_store=None):
        self.omega, self.mode, self.order = omega, mode, order
        self.J, self.P, self.R, self.cell_dofs, self.colours = [], [], [], [], []
        self.A, self.p = [], []
        for l, L in enumerate(levels):
            get = (lambda k: L[k]) if isinstance(L, dict) else (lambda k: getattr(L, k))
            self.J.append(get("J"))
            self.P.append(get("P"))
            self.R.append(get("R"))
            self.cell_dofs.append(np.asarray(get("cell_dofs")))
            self.colours.append(np.asarray(get("colours")))
            if l == 0:
                self.A.append(None)
                self.p.append(None)
            else:
                A, p = setup_level(self.J[l], self.cell_dofs[l])
                if patch_store is not None:
                    A = patch_store(A)
                self.A.append(A)
                self.p.append(p)
        self.coarse_lu = sla.lu_factor(self.J[0].toarray())

    @property
    def n_levels(self):
        return len(self.J)

    def smooth(self, l, b, d, sweeps):
        return smooth(self.J[l], self.A[l], self.cell_dofs[l], self.p[l], b, d, sweeps,
                      self.omega, self.mode, self.order, self.colours[l])

    def coarse_solve(self, b):
        return sla.lu_solve(self.coarse_lu, b)


def vcycle(H, b, nu1=2, nu2=2, level=None):
    """d = V(b) on `level` (default finest), zero initial iterate."""
    l = H.n_levels - 1 if level is None else level
    if l == 0:
        return H.coarse_solve(b)
    d = np.zeros_like(b)
    d = H.smooth(l, b, d, nu1)
    r = b - H.J[l] @ d
    e = vcycle(H, H.R[l] @ r, nu1, nu2, l - 1)
    d = d + H.P[l] @ e
    d = H.smooth(l, b, d, nu2)
    return d
