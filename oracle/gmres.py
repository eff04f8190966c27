"""Restarted GMRES(m) with right preconditioning, FP64 oracle ([S03] as used in Sec. 3).

x = x0 + M Z-combination: the Arnoldi vectors v_j span K_m(J M, r0), the
preconditioned directions z_j = M v_j are kept (flexible form, identical to
plain right preconditioning for a fixed linear M).  Orthogonalisation is
modified Gram-Schmidt; the small least-squares problem is reduced by Givens
rotations, whose last entry |g_{j+1}| is the residual norm of the iterate.
Stopping: |g_{j+1}| <= max(rtol ||b||, atol), happy breakdown, or max_iter
Arnoldi steps (summed over restarts).  Each restart starts from the true
residual b - J x.
"""
import numpy as np
from scipy.linalg import solve_triangular


def gmres(J, b, M, x0=None, restart=30, max_iter=300, rtol=1e-8, atol=0.0):
    """Return (x, iterations, history, converged, true_rel_res).

    J: matrix or callable y = J x; M: callable z = M v (the preconditioner).
    history: residual norms, the initial one then one per Arnoldi step.
    """
    Jop = J if callable(J) else (lambda v: J @ v)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(b)
    tol = max(rtol * bnorm, atol)
    its = 0
    history = []
    converged = False
    while True:
        r = b - Jop(x)
        beta = np.linalg.norm(r)
        if not history:
            history.append(beta)
        if beta <= tol:
            converged = True
            break
        if its >= max_iter:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        stop = False
        for j in range(m):
            Z[j] = M(V[j])
            w = Jop(Z[j])
            for i in range(j + 1):              # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):                  # previous rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            history.append(abs(g[j + 1]))
            j_end = j + 1
            if abs(g[j + 1]) <= tol or hn == 0.0 or its >= max_iter:
                stop = True
                break
            V[j + 1] = w / hn
        y = solve_triangular(H[:j_end, :j_end], g[:j_end])
        x = x + Z[:j_end].T @ y
        if stop and its >= max_iter:
            r = b - Jop(x)
            converged = np.linalg.norm(r) <= tol
            break
    true_rel = np.linalg.norm(b - Jop(x)) / bnorm if bnorm > 0 else 0.0
    return x, its, np.array(history), converged, true_rel
