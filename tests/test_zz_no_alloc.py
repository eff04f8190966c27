"""vanka_smooth_noalloc (the smoothing entry point whose scratch is the library's fixed device array)
against vanka_smooth (scratch in the context's workspace), through the C ABI: the same kernels in the
same order, so the iterates must agree bit for bit.  Two calls in a row, the second on a smaller
level, in the additive and the multiplicative mode; a level too large for the fixed array is refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import build_problem  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_02690_amd as m
    return m


@pytest.mark.parametrize("mode,prec", [("additive", "f64"), ("additive", "f32"), ("multiplicative", "f64")])
def test_noalloc_matches_workspace_smoothing(vk, mode, prec):
    P = build_problem("channel2d_44x8_k1")
    S = vk.Solver([vk.upload_level(L, DEV) for L in P.levels])
    S.vk_set_workspace(prec, 30, device=DEV)
    S.vanka_setup(0.7, mode)
    rng = np.random.default_rng(5)
    L = len(P.levels) - 1
    # first call on the finest level, second on the next (smaller) one
    for l, zero, sweeps in ((L, False, 3), (L - 1, True, 2)):
        n = P.levels[l].n
        b = torch.from_numpy(rng.standard_normal(n)).to(DEV)
        d0 = torch.from_numpy(rng.standard_normal(n)).to(DEV)
        d_ws = d0.clone()
        d_na = d0.clone()
        S.vanka_smooth(l, b, d_ws, sweeps, d_is_zero=zero)
        S.vanka_smooth_noalloc(l, b, d_na, sweeps, d_is_zero=zero)
        torch.cuda.synchronize()
        diff = float((d_ws - d_na).abs().max())
        _say(f"{mode} {prec} level {l} ({n} unknowns): max |diff| {diff:.3e}")
        assert torch.equal(d_ws, d_na)
        assert float(d_na.abs().max()) > 0.0
    S.close()


def test_noalloc_refuses_levels_beyond_the_fixed_scratch(vk):
    """A two-level system whose fine level has 9 437 184 unknowns (its defect alone needs 72 MiB of
    the 64 MiB scratch): J = I, cells of four consecutive DoFs in one colour, an empty transfer.
    vanka_smooth works on it (workspace scratch); vanka_smooth_noalloc refuses it with VK_ERR_ARG."""
    import types
    import scipy.sparse as sp
    n, n0 = 9 * 2 ** 20, 4
    fine = types.SimpleNamespace(J=sp.identity(n, format="csr"), P=sp.csr_matrix((n, n0)),
                                 R=sp.csr_matrix((n0, n)),
                                 cell_dofs=np.arange(n, dtype=np.int32).reshape(-1, 4),
                                 colours=np.zeros(n // 4, dtype=np.int32))
    coarse = types.SimpleNamespace(J=sp.identity(n0, format="csr"), P=None, R=None,
                                   cell_dofs=np.zeros((1, 1), dtype=np.int32), colours=np.zeros(1, dtype=np.int32))
    S = vk.Solver([vk.upload_level(coarse, DEV), vk.upload_level(fine, DEV)])
    S.vk_set_workspace("f64", 4, device=DEV)
    S.vanka_setup(0.7, "additive")
    b = torch.ones(n, dtype=torch.float64, device=DEV)
    d = torch.zeros_like(b)
    S.vanka_smooth(1, b, d, 1, d_is_zero=True)      # J_K = I: one sweep gives d = omega b
    torch.cuda.synchronize()
    assert float((d - 0.7).abs().max()) <= 1e-15
    with pytest.raises(vk.VkError) as e:
        S.vanka_smooth_noalloc(1, b, d, 1)
    assert e.value.status == vk.VK_ERR_ARG and "scratch" in str(e.value)
    S.close()
