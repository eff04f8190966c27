"""Grid-transfer matrices between nested levels (the V-cycle of Sec. 3 needs
them; the paper does not print them).

Prolongation P: level l-1 -> level l is the canonical embedding of nested finite
element spaces: a coarse Q2 field is interpolated at the fine Q2 nodes (1D
weights 3/8, 3/4, -1/8 at the quarter points) and a coarse P1disc field is
rewritten exactly in each child's P1disc basis.  It acts on each Radau time
node separately (only space is coarsened).  Restriction is R = P^T.
"""
import numpy as np
import scipy.sparse as sp


def prolong_1d(n_coarse, refined):
    """Q2 nodal prolongation along one direction (sparse, fine x coarse)."""
    nc_nodes = 2 * n_coarse + 1
    if not refined:
        return sp.identity(nc_nodes, format="csr")
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


def prolongation(coarse, fine):
    """Slab prolongation (scipy CSR, fine.n x coarse.n)."""
    d = fine.d
    ref = refinement(coarse, fine)
    Pn = sp.identity(1, format="csr")
    for i in range(d):                       # first index fastest -> outermost last
        Pn = sp.kron(prolong_1d(coarse.shape[i], ref[i]), Pn, format="csr")
    Pv = sp.kron(Pn, sp.identity(d), format="csr")

    fci = fine.cell_index()
    ccoord = np.stack([fci[:, i] // 2 if ref[i] else fci[:, i] for i in range(d)], axis=1)
    cstr = np.cumprod((1,) + coarse.shape[:-1])
    ccell = (ccoord * cstr).sum(axis=1)
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
    """Fine node id of every coarse Q2 node (coarse nodes are fine nodes)."""
    ref = refinement(coarse, fine)
    ni = coarse.node_index()
    fi = np.stack([ni[:, i] * (2 if ref[i] else 1) for i in range(fine.d)], axis=1)
    fstr = np.cumprod((1,) + fine.node_shape[:-1])
    return (fi * fstr).sum(axis=1)
