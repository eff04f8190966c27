"""FP64 CPU oracle of the Vanka / geometric-multigrid / GMRES solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the solver library never calls
it, and it shares no code with the HIP path.  It is plain NumPy/SciPy in
float64, written from the paper's description (Sec. 3):

  * vanka.py      the patch matrices J_K, their LAPACK inverses, the multiplicity
                  p, the averaged additive Vanka sweep of Eq. 3.4/3.5 and the
                  "overwriting successively" (multiplicative) variant, each in
                  sequential and cell-coloured order;
  * multigrid.py  the coarsest-level direct solve and the V-cycle;
  * gmres.py      restarted GMRES(m) with right preconditioning, modified
                  Gram-Schmidt and Givens rotations;
  * precision.py  round-to-nearest-even storage of the patch inverses in FP32
                  and BF16 (a project extension; parity unpinned, bounded by
                  rounding analysis instead);
  * newton.py     the damped Newton iteration of one slab and the march over
                  consecutive slabs;
  * mlp.py        the multilayer perceptron of the learned initial guess (a
                  project extension): forward, mean-squared-error gradient and
                  Adam, in FP64 with optional BF16 rounding at the stores.
"""
from .vanka import (patch_matrix, patch_matrices, invert_patches, multiplicity, setup_level,
                    additive_sweep, additive_sweep_loop, additive_sweep_correction,
                    multiplicative_sweep, smooth, cell_order)
from .multigrid import OracleHierarchy, vcycle
from .gmres import gmres
from .precision import round_bf16, round_f32
from .newton import newton_slab, march
from . import mlp

__all__ = [
    "patch_matrix", "patch_matrices", "invert_patches", "multiplicity", "setup_level",
    "additive_sweep", "additive_sweep_loop", "additive_sweep_correction",
    "multiplicative_sweep", "smooth", "cell_order",
    "OracleHierarchy", "vcycle", "gmres", "round_bf16", "round_f32",
    "newton_slab", "march", "mlp",
]
