"""Gauss-Radau nodes and the dG(k) time matrices of one slab (Sec. 2, Eq. 2.2;
Sec. 3, the Lagrange basis at the (k+1) Gauss-Radau points before Eq. 3.1).

Reference slab: s in [0, 1], t = t_{n-1} + tau * s.  The right Radau rule
contains the end point s = 1.  A discrete function on the slab is
u(s) = sum_b U_b chi_b(s) with chi_b the Lagrange polynomial at node s_b.

Time matrices (row = test node a, column = trial node b):
  Kt[a, b] = int_0^1 chi_b'(s) chi_a(s) ds + chi_b(0) chi_a(0)
             (time derivative plus the upwind jump at t_{n-1}^+),
  Wt       = diag(w_a)   (the (k+1)-point Radau rule; exact for the mass
             integrand, degree 2k, so the mass-type terms are diagonal),
  c0[a]    = chi_a(0)    (coupling to the previous slab's end value).
The integral in Kt has degree 2k-1 and is evaluated exactly by the rule.
"""
import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def radau_right(k):
    """(k+1)-point right Gauss-Radau rule on [0, 1]: nodes ascending, last = 1.

    Nodes are the roots of P_{k+1}(x) - P_k(x) on [-1, 1] (Legendre P), mapped
    to [0, 1].  Weights make the rule exact for polynomials of degree <= 2k.
    """
    n = k + 1
    if n == 1:
        return np.array([1.0]), np.array([1.0])
    c = np.zeros(n + 1)
    c[n] = 1.0
    c[n - 1] = -1.0
    x = np.sort(np.real(npleg.legroots(c)))
    x[-1] = 1.0
    s = 0.5 * (x + 1.0)
    # exactness for monomials s^0..s^k determines the weights
    V = np.vander(s, n, increasing=True).T
    mom = 1.0 / np.arange(1, n + 1)
    w = np.linalg.solve(V, mom)
    return s, w


def lagrange_at_nodes(nodes):
    """Coefficient arrays (increasing powers) of the Lagrange basis at `nodes`."""
    n = len(nodes)
    polys = []
    for a in range(n):
        p = np.array([1.0])
        for b in range(n):
            if b != a:
                p = nppoly.polymul(p, np.array([-nodes[b], 1.0]) / (nodes[a] - nodes[b]))
        polys.append(p)
    return polys


def dg_time_matrices(k):
    """Return (s, w, Kt, c0) for dG(k) with the right Radau Lagrange basis."""
    s, w = radau_right(k)
    chi = lagrange_at_nodes(s)
    n = k + 1
    Kt = np.zeros((n, n))
    c0 = np.array([nppoly.polyval(0.0, chi[a]) for a in range(n)])
    for a in range(n):
        for b in range(n):
            dchi_b = nppoly.polyder(chi[b])
            # the Radau rule is exact for this degree-(2k-1) integrand and chi_a(s_q) = delta_aq
            Kt[a, b] = w[a] * nppoly.polyval(s[a], dchi_b) + c0[a] * c0[b]
    return s, w, Kt, c0
