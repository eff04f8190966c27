"""Batched solves (independent systems of uneven size and k in one context)
against per-system FP64 oracle runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth.batch import build_batch  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def vk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_02690_amd as m
    return m


@pytest.fixture(scope="module")
def small_batch():
    # 7 systems, meshes 8..32 x 8..24, k in {1,2,3}; hierarchies of 4 and 5 levels
    B = build_batch(n_systems=7, seed=1, nx8=(1, 4), ny8=(1, 3), max_coarse_unknowns=300)
    H = [oracle.OracleHierarchy(h) for h in B.hierarchies]
    return B, H


def make(vk, B, prec="f64"):
    S = vk.Solver([vk.upload_packed_level(L, DEV) for L in B.levels])
    S.vk_set_segments(B.seg_rows)
    S.vk_set_workspace(prec, 30, device=DEV)
    S.vanka_setup(0.7)
    return S


def test_batch_structure(small_batch):
    B, _ = small_batch
    depths = {len(h) for h in B.hierarchies}
    assert len(depths) >= 2, "the test batch must mix hierarchy depths"
    assert len({s["k"] for s in B.systems}) >= 2


def test_batch_vcycle_matches_per_system_oracle(vk, small_batch):
    B, H = small_batch
    S = make(vk, B)
    x = torch.empty(B.levels[-1].n, dtype=torch.float64, device=DEV)
    S.vcycle(torch.from_numpy(B.b).to(DEV), x, 2, 2)
    xg = x.cpu().numpy()
    fin = B.levels[-1]
    for si, (off, n) in fin.rows.items():
        ref = oracle.vcycle(H[si], B.rhs[si], 2, 2)
        err = np.abs(xg[off:off + n] - ref).max() / np.abs(ref).max()
        assert err <= 1e-10, (si, err)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_gmres_matches_per_system_oracle(vk, small_batch, prec):
    B, H = small_batch
    S = make(vk, B, prec)
    x = torch.zeros(B.levels[-1].n, dtype=torch.float64, device=DEV)
    its, rel, conv = S.gmres_solve_batched(torch.from_numpy(B.b).to(DEV), x, restart=30, max_iter=200, rtol=1e-8)
    assert conv
    xg = x.cpu().numpy()
    fin = B.levels[-1]
    order = sorted(fin.rows.items(), key=lambda kv: kv[1][0])
    for seg, (si, (off, n)) in enumerate(order):
        J = B.hierarchies[si][-1].J
        b = B.rhs[si]
        true_rel = np.linalg.norm(b - J @ xg[off:off + n]) / np.linalg.norm(b)
        assert true_rel <= 1e-8 and abs(true_rel - rel[seg]) <= 1e-12
        _, its_o, *_ = oracle.gmres(J, b, lambda v, h=H[si]: oracle.vcycle(h, v, 2, 2))
        assert abs(int(its[seg]) - its_o) <= 1, (si, its[seg], its_o)


def test_batch_zero_rhs_segment(vk, small_batch):
    """A system with b = 0 stays at x = 0 with zero iterations while the others converge."""
    B, _ = small_batch
    S = make(vk, B)
    b = B.b.copy()
    b[B.seg_rows[1]:B.seg_rows[2]] = 0.0
    x = torch.zeros(B.levels[-1].n, dtype=torch.float64, device=DEV)
    its, rel, conv = S.gmres_solve_batched(torch.from_numpy(b).to(DEV), x)
    assert conv and its[1] == 0
    assert float(x[B.seg_rows[1]:B.seg_rows[2]].abs().max()) == 0.0
    assert np.all(its[np.arange(len(its)) != 1] > 0)
