"""Batches of independent systems (many channels of uneven size and k).

Each system is a channel problem of its own mesh, dG order and viscosity; the
channel has height 0.41 and the length that makes its cells square.  For
the solver the batch is packed by depth below the finest level: packed level
D-1-d holds, for every system that has one, its level L_s-1-d, as a
block-diagonal concatenation.  Cells of equal patch width form one group; a
system whose coarsest level sits at depth d contributes a directly solved
diagonal block there instead of cells.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.sparse as sp

from .mesh import StructuredMesh, coarsen_shape
from .problems import H_CHANNEL, build_hierarchy


def batch_shapes(shape, max_coarse_unknowns=1500, k=1):
    """Halve every even direction >= 4 until the level is small or cannot shrink."""
    shapes = [tuple(shape)]
    while True:
        m = StructuredMesh(shapes[0], (1.0,) * len(shape), k)
        if m.n <= max_coarse_unknowns:
            break
        c = coarsen_shape(shapes[0])
        if c == shapes[0]:
            break
        shapes.insert(0, c)
    return shapes


def draw_systems(n_systems=64, seed=0, nx8=(4, 16), ny8=(1, 3)):
    """Mesh n_x = 8 U{4..16}, n_y = 8 U{1..3}, k ~ U{1,2,3}, nu = 10^U(-3,-2)."""
    rng = np.random.default_rng(3000 + seed)
    out = []
    for i in range(n_systems):
        nx = 8 * int(rng.integers(nx8[0], nx8[1] + 1))
        ny = 8 * int(rng.integers(ny8[0], ny8[1] + 1))
        k = int(rng.integers(1, 4))
        nu = float(10.0 ** rng.uniform(-3.0, -2.0))
        out.append(dict(shape=(nx, ny), k=k, nu=nu, seed=100 + 1000 * seed + i))
    return out


@dataclass
class PackedLevel:
    J: sp.csr_matrix
    P: object                      # packed level l-1 -> l (None on level 0)
    R: object
    groups: list                   # dicts: cell_dofs (level-global), colours, n_K
    blocks: np.ndarray             # row offsets of directly solved blocks (n_blocks + 1), or empty
    rows: dict                     # system -> (row offset, n) on this level

    @property
    def n(self):
        return self.J.shape[0]


@dataclass
class Batch:
    systems: List[dict]
    hierarchies: List[list] = field(default_factory=list)   # per system, synth Levels (0 = coarsest)
    rhs: List[np.ndarray] = field(default_factory=list)
    levels: List[PackedLevel] = field(default_factory=list)  # packed, 0 = coarsest
    seg_rows: np.ndarray = None
    b: np.ndarray = None

    @property
    def n_cells_finest(self):
        return sum(h[-1].mesh.n_cells for h in self.hierarchies)


def build_batch(n_systems=64, seed=0, tau=0.01, U=0.3, max_coarse_unknowns=1500, nx8=(4, 16), ny8=(1, 3)):
    systems = draw_systems(n_systems, seed, nx8, ny8)
    B = Batch(systems=systems)
    for s in systems:
        k = s["k"]
        shapes = batch_shapes(s["shape"], max_coarse_unknowns, k)
        # channel length chosen so the finest cells are square
        Lx = H_CHANNEL * s["shape"][0] / s["shape"][1]
        lv = build_hierarchy(d=2, shape=s["shape"], lengths=(Lx, H_CHANNEL), levels=len(shapes), k=k,
                             nu=s["nu"], tau=tau, U=U, seed=s["seed"], shapes=shapes)
        B.hierarchies.append(lv)
        B.rhs.append(np.random.default_rng(2000 + s["seed"]).standard_normal(lv[-1].n))
    D = max(len(h) for h in B.hierarchies)
    packed = []
    for pl in range(D):                       # packed level index, 0 = coarsest
        depth = D - 1 - pl
        rows, blocks, Js = {}, [0], []
        groups = {}
        off = 0
        # systems solved directly at this depth first, so their blocks are contiguous
        present = [si for si, h in enumerate(B.hierarchies) if len(h) - 1 - depth >= 0]
        present.sort(key=lambda si: (len(B.hierarchies[si]) - 1 - depth != 0, si))
        for si in present:
            h = B.hierarchies[si]
            li = len(h) - 1 - depth
            L = h[li]
            rows[si] = (off, L.n)
            Js.append(L.J)
            if li == 0:
                if blocks[-1] != off:
                    raise ValueError("directly solved blocks must be contiguous")
                blocks.append(off + L.n)
            else:
                g = groups.setdefault(L.mesh.n_K, {"cell_dofs": [], "colours": [], "n_K": L.mesh.n_K})
                g["cell_dofs"].append(L.cell_dofs.astype(np.int64) + off)
                g["colours"].append(L.colours)
            off += L.n
        J = sp.block_diag(Js, format="csr")
        J.sort_indices()
        grp = []
        for nK in sorted(groups):
            g = groups[nK]
            grp.append(dict(n_K=nK, cell_dofs=np.concatenate(g["cell_dofs"]).astype(np.int32),
                            colours=np.concatenate(g["colours"]).astype(np.int32)))
        packed.append(PackedLevel(J=J, P=None, R=None, groups=grp,
                                  blocks=np.array(blocks if len(blocks) > 1 else [], dtype=np.int64), rows=rows))
    # transfers between packed levels
    for pl in range(1, D):
        fine, coarse = packed[pl], packed[pl - 1]
        blocks = []
        for si, (f0, fn) in fine.rows.items():
            h = B.hierarchies[si]
            li = len(h) - 1 - (D - 1 - pl)
            if li >= 1:
                c0, cn = coarse.rows[si]
                blocks.append((f0, c0, h[li].P))
        P = sp.csr_matrix((fine.n, coarse.n))
        parts = []
        for f0, c0, Ps in blocks:
            Pc = Ps.tocoo()
            parts.append(sp.coo_matrix((Pc.data, (Pc.row + f0, Pc.col + c0)), shape=(fine.n, coarse.n)))
        P = sum(parts[1:], parts[0]).tocsr() if parts else P
        P.sort_indices()
        R = P.T.tocsr()
        R.sort_indices()
        fine.P, fine.R = P, R
    B.levels = packed
    fin = packed[-1]
    order = sorted(fin.rows.items(), key=lambda kv: kv[1][0])
    B.seg_rows = np.array([0] + [r[0] + r[1] for _, r in order], dtype=np.int64)
    B.b = np.concatenate([B.rhs[si] for si, _ in order])
    return B
