"""Element-wise Vanka smoother, FP64 oracle (Sec. 3, Eq. 3.4 and 3.5a-d).

Notation of the paper: for a cell K the local restriction R_K picks the
components dof(K, mu^) of a global vector, E_K is its transpose (extension by
zero), J_K is the principal submatrix of the level matrix J on the DoFs of K
(all Radau time nodes), and

    S_K(d) = R_K d + omega J_K^{-1} R_K (b - J d)                     (Eq. 3.4)

One smoothing iteration (Eq. 3.5): z = 0, p = 0; for every cell K_i,
y = S_{K_i}(d^{j-1}); z += E_K y; p += 1 on the DoFs of K; then d^j = z / p.

The paper notes that averaging beats "overwriting successively" the DoFs inside
the element loop; that multiplicative form is provided too:
    for K: d[dofs_K] += omega J_K^{-1} (b - J d)[dofs_K].
Cell order is either sequential (K = 0 .. N-1) or coloured (colour by colour,
ascending cell id inside a colour).  In coloured multiplicative order every cell
of a colour uses the iterate left by the previous colour.
"""
import numpy as np
import scipy.sparse as sp


def patch_matrix(J, dofs):
    """J_K[mu^, nu^] = J[dof(K, mu^), dof(K, nu^)]; entries J does not store are 0."""
    dofs = np.asarray(dofs)
    return np.asarray(J[dofs][:, dofs].todense(), dtype=np.float64)


def patch_matrices(J, cell_dofs):
    J = sp.csr_matrix(J)
    return np.stack([patch_matrix(J, cd) for cd in cell_dofs])


def invert_patches(JK):
    """A_K = J_K^{-1} by LAPACK (getrf + getri through numpy.linalg.inv)."""
    return np.linalg.inv(JK)


def multiplicity(cell_dofs, n):
    """p_mu = number of cells whose patch contains DoF mu (Eq. 3.5b count)."""
    return np.bincount(np.asarray(cell_dofs).ravel(), minlength=n).astype(np.float64)


def setup_level(J, cell_dofs):
    """Return (A, p): the patch inverses [N_c, n_K, n_K] and the multiplicity."""
    A = invert_patches(patch_matrices(J, cell_dofs))
    return A, multiplicity(cell_dofs, J.shape[0])


def cell_order(n_cells, order, colours=None):
    if order == "sequential":
        return np.arange(n_cells)
    if order == "coloured":
        return np.argsort(np.asarray(colours), kind="stable")
    raise ValueError(order)


def additive_sweep_loop(J, A, cell_dofs, b, d, omega, order="sequential", colours=None):
    """Eq. 3.5a-d written out cell by cell (reference form for small meshes)."""
    n = J.shape[0]
    z = np.zeros(n)
    p = np.zeros(n)
    r = b - J @ d                       # the defect of d^{j-1}, shared by all S_K
    for K in cell_order(len(cell_dofs), order, colours):
        dofs = cell_dofs[K]
        y = d[dofs] + omega * (A[K] @ r[dofs])         # S_K(d^{j-1})
        for mh in range(len(dofs)):                    # z += E_K y ; p++
            z[dofs[mh]] += y[mh]
            p[dofs[mh]] += 1.0
    return z / p


def additive_sweep(J, A, cell_dofs, b, d, omega, order="sequential", colours=None):
    """Eq. 3.5a-d with the cell loop vectorised; accumulation in the given order."""
    n = J.shape[0]
    ordr = cell_order(len(cell_dofs), order, colours)
    cd = np.asarray(cell_dofs)[ordr]
    r = b - J @ d
    y = d[cd] + omega * np.einsum("kij,kj->ki", A[ordr], r[cd])
    z = np.zeros(n)
    p = np.zeros(n)
    np.add.at(z, cd.ravel(), y.ravel())
    np.add.at(p, cd.ravel(), 1.0)
    return z / p


def additive_sweep_correction(J, A, cell_dofs, p, b, d, omega, order="sequential", colours=None):
    """Same sweep in correction form: d + omega P^{-1} sum_K E_K J_K^{-1} R_K (b - J d).

    Because sum_K E_K R_K d = p * d, this equals Eq. 3.5 exactly in real
    arithmetic.
    """
    ordr = cell_order(len(cell_dofs), order, colours)
    cd = np.asarray(cell_dofs)[ordr]
    r = b - J @ d
    y = np.einsum("kij,kj->ki", A[ordr], r[cd])
    c = np.zeros(J.shape[0])
    np.add.at(c, cd.ravel(), y.ravel())
    return d + omega * c / p


def multiplicative_sweep(J, A, cell_dofs, b, d, omega, order="sequential", colours=None):
    """'Overwriting successively': each cell updates d in place with its local solve."""
    d = np.array(d, dtype=np.float64, copy=True)
    cell_dofs = np.asarray(cell_dofs)
    if order == "sequential":
        J = sp.csr_matrix(J)
        for K in range(len(cell_dofs)):
            dofs = cell_dofs[K]
            rK = b[dofs] - J[dofs] @ d
            d[dofs] += omega * (A[K] @ rK)
        return d
    if order == "coloured":
        colours = np.asarray(colours)
        for c in np.unique(colours):
            cells = np.nonzero(colours == c)[0]
            r = b - J @ d                  # the iterate left by the previous colour
            cd = cell_dofs[cells]
            y = np.einsum("kij,kj->ki", A[cells], r[cd])
            np.add.at(d, cd.ravel(), omega * y.ravel())
        return d
    raise ValueError(order)


def smooth(J, A, cell_dofs, p, b, d, sweeps, omega, mode="additive", order="coloured",
           colours=None):
    """`sweeps` smoothing iterations (J_max of Sec. 3) starting from d."""
    for _ in range(sweeps):
        if mode == "additive":
            d = additive_sweep(J, A, cell_dofs, b, d, omega, order, colours)
        elif mode == "multiplicative":
            d = multiplicative_sweep(J, A, cell_dofs, b, d, omega, order, colours)
        else:
            raise ValueError(mode)
    return d
