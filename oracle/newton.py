"""Damped Newton iteration of one dG(k) slab and the march over slabs, FP64
oracle (Sec. 3: each slab's nonlinear system is solved by Newton's method, the
linear systems by GMRES preconditioned with the multigrid V-cycle).

Damping (the paper names damping without giving the rule): backtracking over
lambda in {1, 1/2, 1/4, 1/8, 1/16}, taking the first lambda with
||F(X + lambda C)|| <= (1 - 1e-4 lambda) ||F(X)|| (the last one if none does).
Stopping: ||F(X)||_2 < tol (absolute, 1e-8).  Each GMRES solve stops at
max(rtol ||F||, atol).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from .gmres import gmres
from .multigrid import OracleHierarchy, vcycle

DAMPING = (1.0, 0.5, 0.25, 0.125, 0.0625)


def newton_slab(residual, levels_of, X0, tol=1e-8, rtol=1e-8, atol=1e-10, max_newton=20, nu=(2, 2)):
    """Solve F(X) = 0 from X0.  residual(X) -> F; levels_of(X) -> multigrid levels of J(X).

    Returns (X, newton iterations, GMRES iterations (total), residual norms)."""
    X = np.array(X0, dtype=np.float64, copy=True)
    F = residual(X)
    nrm = np.linalg.norm(F)
    hist = [nrm]
    its_n = its_g = 0
    while nrm >= tol and its_n < max_newton:
        levels = levels_of(X)
        H = OracleHierarchy(levels)
        C, its, _, conv, _ = gmres(levels[-1].J, -F, lambda v: vcycle(H, v, *nu), rtol=rtol, atol=atol)
        its_g += its
        for lam in DAMPING:
            Xt = X + lam * C
            Ft = residual(Xt)
            nt = np.linalg.norm(Ft)
            if nt <= (1.0 - 1e-4 * lam) * nrm:
                break
        X, F, nrm = Xt, Ft, nt
        hist.append(nrm)
        its_n += 1
    return X, its_n, its_g, hist


def march(problem, n_slabs, guess=None, **kw):
    """Slabs 1..n_slabs of a `synth.march.ChannelMarch`; guess(n, X_prev2, X_prev) -> X0
    (default: the extrapolation of the previous slab).  Returns the slab solutions
    (index 0 = the initial slab) and per-slab (newton, gmres) iteration counts."""
    Xs = [problem.initial_slab()]
    counts = []
    for n in range(1, n_slabs + 1):
        prev = Xs[-1]
        prev2 = Xs[-2] if len(Xs) > 1 else Xs[-1]
        X0 = problem.extrapolate(prev) if guess is None else guess(n, prev2, prev)
        X, its_n, its_g, _ = newton_slab(lambda X: problem.residual(X, prev, n), problem.hierarchy, X0, **kw)
        Xs.append(X)
        counts.append((its_n, its_g))
    return Xs, counts
