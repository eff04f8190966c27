"""Grid-transfer matrices between nested levels (the V-cycle of Sec. 3 needs
them; the paper does not print them).

Prolongation P: level l-1 -> level l is the canonical embedding of nested finite
element spaces: a coarse Q_r field is interpolated at the fine Q_r nodes (for
r = 2 the 1D weights 3/8, 3/4, -1/8 at the quarter points) and a coarse
P_{r-1}disc field is rewritten exactly in each child's basis.  It acts on each
Radau time node separately (only space is coarsened).  Restriction is R = P^T.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import pressure_exponents


def _lagrange_values(t, r):
    """Values of the degree-r Lagrange basis (nodes j / r of [0, 1]) at the points t."""
    nodes = np.arange(r + 1) / r
    val = np.ones((len(t), r + 1))
    for j in range(r + 1):
        for m in range(r + 1):
            if m != j:
                val[:, j] *= (t - nodes[m]) / (nodes[j] - nodes[m])
    return val


def prolong_1d(n_coarse, refined, r=2):
    """Q_r nodal prolongation along one direction (sparse, fine x coarse)."""
    nc_nodes = r * n_coarse + 1
    if not refined:
        return sp.identity(nc_nodes, format="csr")
    if r != 2:
        # fine node j of a coarse cell sits at t = j / (2 r): the coarse basis there
        W = _lagrange_values(np.arange(2 * r) / (2 * r), r)
        W[np.abs(W) < 1e-14] = 0.0
        rows, cols, vals = [], [], []
        for c in range(n_coarse):
            for j in range(2 * r):
                for i in np.nonzero(W[j])[0]:
                    rows.append(2 * r * c + j)
                    cols.append(r * c + i)
                    vals.append(W[j, i])
        rows.append(2 * r * n_coarse)
        cols.append(nc_nodes - 1)
        vals.append(1.0)
        return sp.csr_matrix((vals, (rows, cols)), shape=(2 * r * n_coarse + 1, nc_nodes))
    nf_nodes = 4 * n_coarse + 1
    rows, cols, vals = [], [], []
    for c in range(n_coarse):
        base_f, base_c = 4 * c, 2 * c
        stencil = {
            0: [(0, 1.0)],
            1: [(0, 3 / 8), (1, 3 / 4), (2, -1 / 8)],
            2: [(1, 1.0)],
            3: [(0, -1 / 8), (1, 3 / 4), (2, 3 / 8)],
        }
        for f_off, taps in stencil.items():
            for c_off, w in taps:
                rows.append(base_f + f_off)
                cols.append(base_c + c_off)
                vals.append(w)
    rows.append(nf_nodes - 1)
    cols.append(nc_nodes - 1)
    vals.append(1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf_nodes, nc_nodes))


def refinement(coarse, fine):
    r = []
    for nc, nf in zip(coarse.shape, fine.shape):
        if nf == 2 * nc:
            r.append(True)
        elif nf == nc:
            r.append(False)
        else:
            raise ValueError("levels are not nested")
    return r


def child_pressure_maps(d, r, ref):
    """T[sigma] (m x m): a coarse cell's P_{r-1} coefficients -> those of its child sigma (bit i of
    sigma: upper half along refined direction i), the same polynomial in the child's reference
    coordinates x^_c = (x^_f + 2 sigma_i - 1) / 2 along refined directions (x^_f otherwise)."""
    ex = np.array(pressure_exponents(d, r))
    m = len(ex)
    pts = np.random.default_rng(0).uniform(-1.0, 1.0, size=(4 * m, d))
    Vf = np.prod(pts[:, None, :] ** ex[None, :, :], axis=2)
    maps = {}
    for sigma in range(1 << d):
        xc = pts.copy()
        for i in range(d):
            if ref[i]:
                xc[:, i] = (pts[:, i] + 2.0 * ((sigma >> i) & 1) - 1.0) / 2.0
        Vc = np.prod(xc[:, None, :] ** ex[None, :, :], axis=2)
        T = np.linalg.lstsq(Vf, Vc, rcond=None)[0]
        T[np.abs(T) < 1e-12] = 0.0
        maps[sigma] = T
    return maps


def prolongation(coarse, fine):
    """Slab prolongation (scipy CSR, fine.n x coarse.n)."""
    d = fine.d
    r = fine.r
    if coarse.r != r:
        raise ValueError("levels of one hierarchy share the velocity degree")
    ref = refinement(coarse, fine)
    Pn = sp.identity(1, format="csr")
    for i in range(d):                       # first index fastest -> outermost last
        Pn = sp.kron(prolong_1d(coarse.shape[i], ref[i], r), Pn, format="csr")
    Pv = sp.kron(Pn, sp.identity(d), format="csr")

    fci = fine.cell_index()
    ccoord = np.stack([fci[:, i] // 2 if ref[i] else fci[:, i] for i in range(d)], axis=1)
    cstr = np.cumprod((1,) + coarse.shape[:-1])
    ccell = (ccoord * cstr).sum(axis=1)
    if r != 2:
        m = fine.n_pmodes
        maps = child_pressure_maps(d, r, ref)
        sig = sum(((fci[:, i] % 2) << i) if ref[i] else 0 * fci[:, i] for i in range(d))
        rows, cols, vals = [], [], []
        for f in range(fine.n_cells):
            T = maps[int(sig[f])]
            pi, qi = np.nonzero(T)
            rows.append(f * m + pi)
            cols.append(ccell[f] * m + qi)
            vals.append(T[pi, qi])
        Pp = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(fine.n_pres, coarse.n_pres))
        Ps = sp.block_diag([Pv, Pp], format="csr")
        P = sp.kron(sp.identity(fine.n_time), Ps, format="csr")
        P.sum_duplicates()
        P.sort_indices()
        return P
    rows, cols, vals = [], [], []
    nq = d + 1
    for i in range(d):
        sig = np.where(fci[:, i] % 2 == 1, 1.0, -1.0) if ref[i] else np.zeros(fine.n_cells)
        # constant coefficient picks up sigma_i / 2 of the coarse slope
        rows.append(np.arange(fine.n_cells) * nq)
        cols.append(ccell * nq + 1 + i)
        vals.append(sig / 2.0)
        rows.append(np.arange(fine.n_cells) * nq + 1 + i)
        cols.append(ccell * nq + 1 + i)
        vals.append(np.full(fine.n_cells, 0.5 if ref[i] else 1.0))
    rows.append(np.arange(fine.n_cells) * nq)
    cols.append(ccell * nq)
    vals.append(np.ones(fine.n_cells))
    Pp = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(fine.n_pres, coarse.n_pres))
    Pp.eliminate_zeros()
    Ps = sp.block_diag([Pv, Pp], format="csr")
    P = sp.kron(sp.identity(fine.n_time), Ps, format="csr")
    P.sum_duplicates()
    P.sort_indices()
    return P


def inject_nodes(coarse, fine):
    """Fine node id of every coarse node (coarse nodes are fine nodes)."""
    ref = refinement(coarse, fine)
    ni = coarse.node_index()
    fi = np.stack([ni[:, i] * (2 if ref[i] else 1) for i in range(fine.d)], axis=1)
    fstr = np.cumprod((1,) + fine.node_shape[:-1])
    return (fi * fstr).sum(axis=1)
