"""Parity at the workloads' full sizes, in the configuration bench.py times.

* 176 x 32 dG(2) channel (188 358 unknowns, 5 levels): the whole oracle still runs in seconds, so the
  V-cycle is compared element by element (1e-10) and GMRES counts within +-1.
* 100 x 16 x 16 dG(1) box (1 518 134 unknowns, n_K = 170): sampled outputs the oracle computes one by
  one (patch inverses of sampled cells; the sweep update of sampled DoFs from Eq. 3.5 with the inverses
  of the cells that contain them), and GMRES's true residual (a property at any size).
* The 64-system batch: every system's true residual, and the iteration counts of the two smallest
  systems against their own oracle solves.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
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


def solver(vk, levels, prec):
    S = vk.Solver([vk.upload_level(L, DEV) for L in levels])
    S.vk_set_workspace(prec, 30, device=DEV)
    S.vanka_setup(0.7, "additive")
    S.vk_autotune(3)
    return S


def test_channel_176x32_k2_full(vk):
    _say("build channel2d_176x32_k2")
    P = build_problem("channel2d_176x32_k2")
    H = oracle.OracleHierarchy(P.levels)
    b = torch.from_numpy(P.b).to(DEV)
    S = solver(vk, P.levels, "f64")
    x = torch.empty_like(b)
    S.vcycle(b, x, 2, 2)
    ref = oracle.vcycle(H, P.b, 2, 2)
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    _, its_o, *_ = oracle.gmres(P.finest.J, P.b, lambda v: oracle.vcycle(H, v, 2, 2))
    for prec in ("f64", "f32"):
        S2 = S if prec == "f64" else solver(vk, P.levels, prec)
        x = torch.zeros_like(b)
        its, rel, _, ok = S2.gmres_solve(b, x, rtol=1e-8)
        true_rel = np.linalg.norm(P.b - P.finest.J @ x.cpu().numpy()) / np.linalg.norm(P.b)
        assert ok and true_rel <= 1e-8 and abs(its - its_o) <= 1, (prec, its, its_o, true_rel)
        S2.close()


def test_box3d_full_sampled(vk):
    _say("build box3d_100x16x16_k1")
    P = build_problem("box3d_100x16x16_k1")
    F = P.finest
    S = solver(vk, P.levels, "f64")
    rng = np.random.default_rng(11)
    L = len(P.levels) - 1
    # sampled patch inverses on the finest and the next level
    for l, n_s in ((L, 24), (L - 1, 12)):
        lv = P.levels[l]
        cells = np.sort(rng.choice(lv.mesh.n_cells, n_s, replace=False))
        nK = lv.mesh.n_K
        out = torch.empty((1, nK, nK), dtype=torch.float64, device=DEV)
        for K in cells:
            S.vk_get_patch_inverses(l, int(K), 1, out)
            ref = np.linalg.inv(oracle.patch_matrix(lv.J, lv.cell_dofs[K]))
            assert np.abs(out[0].cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max(), (l, K)
    # one additive sweep from a nonzero iterate: d'_mu = d_mu + omega / p_mu sum_{K ni mu} (A_K r_K)[mu]
    d0 = rng.standard_normal(F.n)
    d = torch.from_numpy(d0).to(DEV)
    b = torch.from_numpy(P.b).to(DEV)
    S.vanka_smooth(L, b, d, 1, d_is_zero=False)
    got = d.cpu().numpy()
    r = P.b - F.J @ d0
    cd = F.cell_dofs
    p = oracle.multiplicity(cd, F.n)
    mus = rng.choice(F.n, 40, replace=False)
    for mu in mus:
        cells = np.nonzero((cd == mu).any(axis=1))[0]
        z = 0.0
        for K in cells:
            A = np.linalg.inv(oracle.patch_matrix(F.J, cd[K]))
            loc = int(np.nonzero(cd[K] == mu)[0][0])
            z += (A @ r[cd[K]])[loc]
        ref = d0[mu] + 0.7 * z / p[mu]
        assert abs(got[mu] - ref) <= 1e-10 * max(1.0, abs(ref)), (mu, got[mu], ref)
    # GMRES to 1e-8: the true residual on the host
    x = torch.zeros_like(b)
    its, rel, _, ok = S.gmres_solve(b, x, rtol=1e-8)
    true_rel = np.linalg.norm(P.b - F.J @ x.cpu().numpy()) / np.linalg.norm(P.b)
    _say(f"box3d gmres {its} its, true rel {true_rel:.2e}")
    assert ok and true_rel <= 1e-8 and abs(true_rel - rel) <= 1e-12
    S.close()


def test_batch64_full(vk):
    from synth.batch import build_batch
    _say("build batch64 seed 0")
    B = build_batch(64, seed=0)
    S = vk.Solver([vk.upload_packed_level(L, DEV) for L in B.levels])
    S.vk_set_segments(B.seg_rows)
    S.vk_set_workspace("f32", 30, device=DEV)
    S.vanka_setup(0.7)
    S.vk_autotune(3)
    S.vk_set_graphs(True)
    x = torch.zeros(B.levels[-1].n, dtype=torch.float64, device=DEV)
    its, rel, conv = S.gmres_solve_batched(torch.from_numpy(B.b).to(DEV), x, rtol=1e-8)
    assert conv
    xg = x.cpu().numpy()
    order = sorted(B.levels[-1].rows.items(), key=lambda kv: kv[1][0])
    for seg, (si, (off, n)) in enumerate(order):
        J = B.hierarchies[si][-1].J
        true_rel = np.linalg.norm(B.rhs[si] - J @ xg[off:off + n]) / np.linalg.norm(B.rhs[si])
        assert true_rel <= 1e-8 and abs(true_rel - rel[seg]) <= 1e-12, (si, true_rel, rel[seg])
    sizes = [B.hierarchies[si][-1].n for si, _ in order]
    for seg in np.argsort(sizes)[:2]:
        si = order[seg][0]
        Hs = oracle.OracleHierarchy(B.hierarchies[si])
        _, its_o, *_ = oracle.gmres(B.hierarchies[si][-1].J, B.rhs[si], lambda v: oracle.vcycle(Hs, v, 2, 2))
        assert abs(int(its[seg]) - its_o) <= 1, (si, its[seg], its_o)
    S.close()
