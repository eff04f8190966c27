"""Parity at the workloads' full sizes, in the configuration bench.py times.

* 176 x 32 dG(2) channel (188 358 unknowns, 5 levels): the whole oracle still runs in seconds, so the
  V-cycle is compared element by element (1e-10); GMRES counts within +-1 of the oracle for FP64, FP32
  and BF16 patch inverses and for the paper's four-plus-four smoothing iterations.
* 100 x 16 x 16 dG(1) box (1 518 134 unknowns, n_K = 170): sampled outputs the oracle computes one by
  one (patch inverses of sampled cells; the sweep update of sampled DoFs from Eq. 3.5 with the inverses
  of the cells that contain them); the 4-level V-cycle at 2 000 sampled entries and its 2-norm; GMRES
  counts within +-1 for FP64 and FP32 inverses with true residuals <= 1e-8.
* The 64-system batch: every system's true residual and iteration count (+-1).

The oracle's counts, V-cycle sample and norms at these sizes take minutes to hours on the host, so they
come from tests/golden/oracle_counts.json, written by tests/golden/make_oracle_counts.py, which calls only
the oracle and the seeded input generators.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth import build_problem  # noqa: E402

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_counts.json")


def golden(key):
    with open(GOLDEN) as f:
        ent = json.load(f)["entries"]
    if key not in ent:
        pytest.fail(f"{key} missing from {GOLDEN}: run tests/golden/make_oracle_counts.py")
    return ent[key]


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
    assert its_o == golden("channel2d_176x32_k2/f64/nu22")["iters"]
    for prec in ("f64", "f32", "bf16"):
        S2 = S if prec == "f64" else solver(vk, P.levels, prec)
        for nu in ((2, 2), (4, 4)):
            key = f"channel2d_176x32_k2/{prec}/nu{nu[0]}{nu[1]}"
            if nu == (4, 4) and prec == "bf16":
                continue
            its_g = golden(key)["iters"]
            x = torch.zeros_like(b)
            its, rel, _, ok = S2.gmres_solve(b, x, rtol=1e-8, nu_pre=nu[0], nu_post=nu[1])
            true_rel = np.linalg.norm(P.b - P.finest.J @ x.cpu().numpy()) / np.linalg.norm(P.b)
            _say(f"{key}: {its} its (oracle {its_g}), true rel {true_rel:.2e}")
            assert ok and true_rel <= 1e-8 and abs(its - its_g) <= 1, (key, its, its_g, true_rel)
        if S2 is not S:
            S2.close()


def test_grouped_csr_products_176x32(vk):
    """The grouped CSR of the 176 x 32 channel's finest J (10.5 M nonzeros): the products y = J x and
    y = z - J x equal scipy's CSR products and the library's own CSR products to rounding, on the
    finest level and the next one."""
    P = build_problem("channel2d_176x32_k2")
    S = vk.Solver([vk.upload_level(L, DEV) for L in P.levels])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vanka_setup(0.7, "additive")
    rng = np.random.default_rng(21)
    for l in (len(P.levels) - 1, len(P.levels) - 2):
        J = P.levels[l].J
        if J.nnz < 4 << 20:
            assert S.vk_spmv_format(l) == 0
            continue
        assert S.vk_spmv_format(l) > 0, l
        x = rng.standard_normal(J.shape[0])
        z = rng.standard_normal(J.shape[0])
        xt = torch.from_numpy(x).to(DEV)
        zt = torch.from_numpy(z).to(DEV)
        y = torch.empty_like(xt)
        ref = J @ x
        ref2 = z - J @ x
        # the library's choice of lanes per group, then every count (64: one group per wavefront)
        for lanes in (1, 4, 8, 16, 32, 64):
            S.vk_set_spmv_format(lanes)
            assert lanes == 1 or S.vk_spmv_format(l) == lanes
            S.vk_spmv(l, xt, y)
            assert np.abs(y.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max(), lanes
            S.vk_spmv(l, xt, y, alpha=-1.0, beta=1.0, z=zt)
            assert np.abs(y.cpu().numpy() - ref2).max() <= 1e-13 * np.abs(ref2).max(), lanes
        for bad in (2, 3, 128, -1):
            with pytest.raises(vk.VkError) as e:
                S.vk_set_spmv_format(bad)
            assert e.value.status == vk.VK_ERR_ARG
        S.vk_set_spmv_format(0)
        assert S.vk_spmv_format(l) == 0
        y2 = torch.empty_like(xt)
        S.vk_spmv(l, xt, y2)
        assert np.abs(y2.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
        S.vk_set_spmv_format(1)
    S.close()


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
    # the finest J's products in the grouped CSR with one group per wavefront (the layout the
    # autotuned solve picks for these rows; J is beyond the cache, so its streams load
    # non-temporally) and with the library's own choice of lanes
    xs = rng.standard_normal(F.n)
    zs = rng.standard_normal(F.n)
    xt, zt = torch.from_numpy(xs).to(DEV), torch.from_numpy(zs).to(DEV)
    ys = torch.empty_like(xt)
    ref = F.J @ xs
    for lanes in (64, 1):
        S.vk_set_spmv_format(lanes)
        assert S.vk_spmv_format(L) > 0 and (lanes == 1 or S.vk_spmv_format(L) == lanes)
        S.vk_spmv(L, xt, ys, alpha=-1.0, beta=1.0, z=zt)
        err = np.abs(ys.cpu().numpy() - (zs - ref)).max() / np.abs(zs - ref).max()
        _say(f"box3d grouped J product, lanes {S.vk_spmv_format(L)}: max rel err {err:.2e}")
        assert err <= 1e-13, lanes
    del xt, zt, ys
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
    # the 4-level V-cycle from b at the oracle's sampled entries (relative to the oracle's max |V(b)|)
    ref = golden("box3d_100x16x16_k1/f64/vcycle22_sample")
    v = torch.empty_like(b)
    S.vcycle(b, v, 2, 2)
    vg = v.cpu().numpy()
    idx = np.asarray(ref["indices"])
    err = np.abs(vg[idx] - np.asarray(ref["values"])).max() / ref["max_abs"]
    _say(f"box3d V-cycle sample: max rel err {err:.2e}")
    assert err <= 1e-10
    assert abs(np.linalg.norm(vg) - ref["norm2"]) <= 1e-10 * ref["norm2"]
    assert abs(np.abs(vg).max() - ref["max_abs"]) <= 1e-10 * ref["max_abs"]
    # GMRES to 1e-8 with FP64 and FP32 inverses: counts against the oracle's, true residual on the host
    for prec in ("f64", "f32"):
        S2 = S if prec == "f64" else solver(vk, P.levels, prec)
        its_g = golden(f"box3d_100x16x16_k1/{prec}/nu22")["iters"]
        x = torch.zeros_like(b)
        its, rel, _, ok = S2.gmres_solve(b, x, rtol=1e-8)
        true_rel = np.linalg.norm(P.b - F.J @ x.cpu().numpy()) / np.linalg.norm(P.b)
        _say(f"box3d gmres {prec}: {its} its (oracle {its_g}), true rel {true_rel:.2e}")
        assert ok and true_rel <= 1e-8 and abs(true_rel - rel) <= 1e-12
        assert abs(its - its_g) <= 1, (prec, its, its_g)
        S2.close()


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
    # every system's count against the oracle's solve of that system alone (FP32-rounded inverses)
    ref = golden("batch64_seed0/f32/nu22")
    bad = [(si, int(its[seg]), ref[str(si)]["iters"]) for seg, (si, _) in enumerate(order)
           if abs(int(its[seg]) - ref[str(si)]["iters"]) > 1]
    _say(f"batch64 counts {int(its.min())}..{int(its.max())}; outside +-1 of the oracle: {bad}")
    assert not bad
    # the smallest system once more against a fresh oracle solve (pins the golden file itself)
    sizes = [B.hierarchies[si][-1].n for si, _ in order]
    seg = int(np.argmin(sizes))
    si = order[seg][0]
    Hs = oracle.OracleHierarchy(B.hierarchies[si], patch_store=oracle.round_f32)
    _, its_o, *_ = oracle.gmres(B.hierarchies[si][-1].J, B.rhs[si], lambda v: oracle.vcycle(Hs, v, 2, 2))
    assert its_o == ref[str(si)]["iters"]
    S.close()
