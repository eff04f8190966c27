"""GPU parity of libvk against the FP64 CPU oracle, through the C ABI.

Tolerances: FP64 paths 1e-10 relative (max-norm); patch inverses and the coarse
inverse relative to their conditioning; FP32/BF16 patch storage 2e-5 against
the oracle with identically rounded inverses (FP32 accumulation over n_K <= 84
terms: n_K * 2^-24 ~ 5e-6, times a safety factor of 4); GMRES counts within
+-1 of the oracle and a true relative residual <= 1e-8.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from synth import build_problem  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_02690_amd as m
    return m


DEV = "cuda:0"

CASES = {
    # name: (config, overrides)
    "cfg0": ("channel2d_44x8_k1", {}),
    "ragged_k2": ("channel2d_44x8_k1", dict(shape=(10, 6), levels=2, k=2)),
    "k3": ("channel2d_44x8_k1", dict(shape=(12, 4), levels=2, k=3)),
    # 3D box, Q2/P1disc hexahedra, dG(1): n_K = 170 (the box's patch width) on a small mesh
    "box3d": ("box3d_100x16x16_k1", dict(shape=(8, 4, 4), levels=2)),
    # the other time degrees of the robustness-in-k study: 2D n_K = 21 (dG(0)) and 105 (dG(4)),
    # 3D n_K = 85 (dG(0)) and 255 (dG(2), patches inverted through global memory)
    "k0": ("channel2d_44x8_k1", dict(shape=(12, 4), levels=2, k=0)),
    "k4": ("channel2d_44x8_k1", dict(shape=(12, 4), levels=2, k=4)),
    "box3d_k0": ("box3d_100x16x16_k1", dict(shape=(8, 4, 4), levels=2, k=0)),
    "box3d_k2": ("box3d_100x16x16_k1", dict(shape=(4, 2, 2), levels=2, k=2)),
    # (Q4)^2 x P3disc, the element of the paper's 2D study: n_K = 60 (k + 1)
    "r4_k0": ("channel2d_44x8_k1", dict(shape=(8, 4), levels=2, k=0, r=4)),
    "r4_k1": ("channel2d_44x8_k1", dict(shape=(8, 4), levels=2, k=1, r=4)),
    "r4_k2": ("channel2d_44x8_k1", dict(shape=(8, 4), levels=2, k=2, r=4)),
    # wider than any register-resident kernel: the blocked Gauss-Jordan path
    "r4_k3": ("channel2d_44x8_k1", dict(shape=(8, 4), levels=2, k=3, r=4)),
    # the widest patch of the study: (Q4)^2 x P3disc dG(4), n_K = 300
    "r4_k4": ("channel2d_44x8_k1", dict(shape=(8, 4), levels=2, k=4, r=4)),
}

_cache = {}


def problem(name):
    if name not in _cache:
        cfg, over = CASES[name] if name in CASES else (name, {})
        P = build_problem(cfg, **over)
        _cache[name] = (P, oracle.OracleHierarchy(P.levels))
    return _cache[name]


def make_solver(vk, P, prec="f64", mode="additive", restart=30):
    S = vk.Solver([vk.upload_level(L, DEV) for L in P.levels])
    S.vk_set_workspace(prec, restart, device=DEV)
    S.vanka_setup(0.7, mode)
    return S


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("case", list(CASES))
def test_spmv(vk, case):
    P, _ = problem(case)
    S = make_solver(vk, P)
    rng = np.random.default_rng(1)
    for l, L in enumerate(P.levels):
        x = rng.standard_normal(L.n)
        y = torch.empty(L.n, dtype=torch.float64, device=DEV)
        S.vk_spmv(l, t(x), y)
        assert rel(y.cpu().numpy(), L.J @ x) <= 1e-13
        z = rng.standard_normal(L.n)
        S.vk_spmv(l, t(x), y, alpha=-1.0, beta=1.0, z=t(z))
        assert rel(y.cpu().numpy(), z - L.J @ x) <= 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_patch_inverses(vk, case):
    P, H = problem(case)
    S = make_solver(vk, P)
    for l in range(1, len(P.levels)):
        nc, nK = P.levels[l].mesh.n_cells, P.levels[l].mesh.n_K
        out = torch.empty((nc, nK, nK), dtype=torch.float64, device=DEV)
        S.vk_get_patch_inverses(l, 0, nc, out)
        got = out.cpu().numpy()
        err = np.abs(got - H.A[l]).max(axis=(1, 2)) / np.abs(H.A[l]).max(axis=(1, 2))
        assert err.max() <= 1e-10, (l, err.max())


@pytest.mark.parametrize("case", ["cfg0"])
def test_coarse_inverse(vk, case):
    P, _ = problem(case)
    S = make_solver(vk, P)
    J0 = P.levels[0].J.toarray()
    n0 = J0.shape[0]
    out = torch.empty((n0, n0), dtype=torch.float64, device=DEV)
    S.vk_get_coarse_inverse(out)
    ref = np.linalg.inv(J0)
    kappa = np.linalg.cond(J0)
    assert rel(out.cpu().numpy(), ref) <= 100 * kappa * np.finfo(float).eps


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("zero", [False, True])
def test_smooth_additive(vk, case, zero):
    P, H = problem(case)
    S = make_solver(vk, P)
    rng = np.random.default_rng(2)
    for l in range(1, len(P.levels)):
        L = P.levels[l]
        b = rng.standard_normal(L.n)
        d0 = np.zeros(L.n) if zero else rng.standard_normal(L.n)
        d = t(d0)
        _say(f"smooth additive {case} level {l} zero={zero}")
        S.vanka_smooth(l, t(b), d, 2, d_is_zero=zero)
        ref = H.smooth(l, b, d0, 2)
        assert rel(d.cpu().numpy(), ref) <= 1e-10, (l, rel(d.cpu().numpy(), ref))


@pytest.mark.parametrize("case", list(CASES))
def test_smooth_multiplicative(vk, case):
    P, _ = problem(case)
    Hm = oracle.OracleHierarchy(P.levels, mode="multiplicative", order="coloured")
    S = make_solver(vk, P, mode="multiplicative")
    rng = np.random.default_rng(3)
    for l in range(1, len(P.levels)):
        L = P.levels[l]
        b = rng.standard_normal(L.n)
        d0 = rng.standard_normal(L.n)
        d = t(d0)
        _say(f"smooth multiplicative {case} level {l}")
        S.vanka_smooth(l, t(b), d, 2)
        ref = Hm.smooth(l, b, d0, 2)
        assert rel(d.cpu().numpy(), ref) <= 1e-10


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("nu", [(2, 2), (1, 0), (0, 1)])
def test_vcycle(vk, case, nu):
    P, H = problem(case)
    S = make_solver(vk, P)
    b = np.random.default_rng(4).standard_normal(P.finest.n)
    x = torch.empty(P.finest.n, dtype=torch.float64, device=DEV)
    _say(f"vcycle {case} nu={nu}")
    S.vcycle(t(b), x, *nu)
    ref = oracle.vcycle(H, b, *nu)
    assert rel(x.cpu().numpy(), ref) <= 1e-10


@pytest.mark.parametrize("case", list(CASES))
def test_gmres(vk, case):
    P, H = problem(case)
    S = make_solver(vk, P)
    b = P.b
    x = torch.zeros(P.finest.n, dtype=torch.float64, device=DEV)
    _say(f"gmres {case}")
    its, relres, hist, ok = S.gmres_solve(t(b), x, restart=30, max_iter=200, rtol=1e-8)
    xo, its_o, hist_o, ok_o, rel_o = oracle.gmres(P.finest.J, b, lambda v: oracle.vcycle(H, v, 2, 2))
    xg = x.cpu().numpy()
    true_rel = np.linalg.norm(b - P.finest.J @ xg) / np.linalg.norm(b)
    assert ok and ok_o
    assert abs(its - its_o) <= 1, (its, its_o)
    assert true_rel <= 1e-8 and abs(true_rel - relres) <= 1e-12
    assert np.all(np.diff(hist) <= 0)
    np.testing.assert_allclose(hist[: min(len(hist), len(hist_o)) - 1],
                               hist_o[: min(len(hist), len(hist_o)) - 1], rtol=1e-6)


@pytest.mark.parametrize("prec,store,tol_rounded,tol_f64", [("f32", oracle.round_f32, 2e-5, 1e-5),
                                                           ("bf16", oracle.round_bf16, 2e-5, 2e-2)])
def test_mixed_precision_sweep(vk, prec, store, tol_rounded, tol_f64):
    P, H = problem("cfg0")
    Hr = oracle.OracleHierarchy(P.levels, patch_store=store)
    S = make_solver(vk, P, prec=prec)
    rng = np.random.default_rng(5)
    for l in range(1, len(P.levels)):
        L = P.levels[l]
        nc, nK = L.mesh.n_cells, L.mesh.n_K
        out = torch.empty((nc, nK, nK), dtype=torch.float64, device=DEV)
        S.vk_get_patch_inverses(l, 0, nc, out)
        ulp = 2.0 ** -24 if prec == "f32" else 2.0 ** -8
        # both sides round an FP64 inverse; the two FP64 inverses agree to 1e-10 of the
        # cell's largest entry (see test_patch_inverses), so the stored values agree to
        # one rounding step plus that
        a = np.abs(out.cpu().numpy() - Hr.A[l])
        cell_max = np.abs(H.A[l]).max(axis=(1, 2), keepdims=True)
        assert np.all(a <= 2 * ulp * np.abs(H.A[l]) + 1e-10 * cell_max), l
        b = rng.standard_normal(L.n)
        d0 = rng.standard_normal(L.n)
        d = t(d0)
        S.vanka_smooth(l, t(b), d, 1)
        got = d.cpu().numpy()
        assert rel(got, Hr.smooth(l, b, d0, 1)) <= tol_rounded
        assert rel(got, H.smooth(l, b, d0, 1)) <= tol_f64


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_precision_gmres(vk, prec):
    P, H = problem("cfg0")
    S = make_solver(vk, P, prec=prec)
    x = torch.zeros(P.finest.n, dtype=torch.float64, device=DEV)
    its, relres, hist, ok = S.gmres_solve(t(P.b), x, restart=30, max_iter=200, rtol=1e-8)
    true_rel = np.linalg.norm(P.b - P.finest.J @ x.cpu().numpy()) / np.linalg.norm(P.b)
    _say(f"gmres {prec}: {its} its, true rel {true_rel:.2e}")
    assert ok and true_rel <= 1e-8


def test_error_paths(vk):
    P, _ = problem("cfg0")
    S = make_solver(vk, P)
    b = t(P.b)
    x = torch.zeros_like(b)
    # b = 0 -> x = 0, zero iterations
    x.fill_(1.0)
    its, relres, hist, ok = S.gmres_solve(torch.zeros_like(b), x)
    assert ok and its == 0 and float(x.abs().max()) == 0.0
    # max_iter = 1 -> no convergence, reported
    x.zero_()
    its, relres, hist, ok = S.gmres_solve(b, x, max_iter=1, raise_on_noconv=False)
    assert not ok and its == 1 and relres > 1e-8
    with pytest.raises(vk.VkError) as e:
        S.gmres_solve(b, x, max_iter=1)
    assert e.value.status == vk.VK_ERR_NOCONV
    # level 0 is solved directly, not smoothed
    with pytest.raises(vk.VkError) as e:
        S.vanka_smooth(0, b[:P.levels[0].n], x[:P.levels[0].n], 1)
    assert e.value.status == vk.VK_ERR_ARG
    # restart larger than the workspace's
    with pytest.raises(vk.VkError):
        S.gmres_solve(b, x, restart=40)


def test_state_and_workspace_errors(vk):
    P, _ = problem("cfg0")
    S = vk.Solver([vk.upload_level(L, DEV) for L in P.levels])
    b = t(P.b)
    x = torch.zeros_like(b)
    with pytest.raises(vk.VkError) as e:
        S.vcycle(b, x)
    assert e.value.status == vk.VK_ERR_WORKSPACE
    need = S.vk_workspace_bytes("f64", 30)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    import ctypes
    st = vk.lib().vk_set_workspace(S.ctx, ctypes.c_void_p(ws.data_ptr()), need - 4096, vk.VK_F64, 30)
    assert st == vk.VK_ERR_WORKSPACE
    S.vk_set_workspace("f64", 30, device=DEV)
    with pytest.raises(vk.VkError) as e:
        S.vcycle(b, x)
    assert e.value.status == vk.VK_ERR_STATE


def test_singular_patch_reported(vk):
    P = build_problem("channel2d_44x8_k1", shape=(8, 4), levels=2)
    L = P.finest
    J = L.J.tolil()
    cell = 5
    pdof = int(L.cell_dofs[cell][18])   # a pressure DoF: it belongs to this cell only
    J[pdof, :] = 0.0
    J = J.tocsr()
    J.eliminate_zeros()
    J.sort_indices()
    L.J = J
    S = vk.Solver([vk.upload_level(Lv, DEV) for Lv in P.levels])
    S.vk_set_workspace("f64", 30, device=DEV)
    with pytest.raises(vk.VkError) as e:
        S.vanka_setup(0.7)
    assert e.value.status == vk.VK_ERR_SINGULAR
    assert e.value.bad_level == 1 and e.value.bad_cell == cell


def test_singular_wide_patch_reported(vk):
    """A singular 255-wide patch (3D dG(2)), inverted by the blocked kernels, names its cell."""
    P = build_problem("box3d_100x16x16_k1", shape=(4, 2, 2), levels=2, k=2)
    L = P.finest
    assert L.mesh.n_K == 255
    J = L.J.tolil()
    cell = 5
    pdof = int(L.cell_dofs[cell][81])   # the first pressure DoF of time node 0: this cell's only
    J[pdof, :] = 0.0
    J = J.tocsr()
    J.eliminate_zeros()
    J.sort_indices()
    L.J = J
    S = vk.Solver([vk.upload_level(Lv, DEV) for Lv in P.levels])
    S.vk_set_workspace("f32", 30, device=DEV)
    with pytest.raises(vk.VkError) as e:
        S.vanka_setup(0.7)
    assert e.value.status == vk.VK_ERR_SINGULAR
    assert e.value.bad_level == 1 and e.value.bad_cell == cell
    S.close()


@pytest.mark.parametrize("variant", [0, 2, 3])
def test_singular_170_patch_reported(vk, variant):
    """A singular 170-wide patch (3D dG(1)) names its cell, on the matrix cores (variant 0 through the
    patch entry map, variant 3 through the LDS hash) and on the vector unit (variant 2)."""
    P = build_problem("box3d_100x16x16_k1", shape=(4, 2, 2), levels=2, k=1)
    L = P.finest
    assert L.mesh.n_K == 170
    J = L.J.tolil()
    cell = 5
    pdof = int(L.cell_dofs[cell][81])   # the first pressure DoF of time node 0: this cell's only
    J[pdof, :] = 0.0
    J = J.tocsr()
    J.eliminate_zeros()
    J.sort_indices()
    L.J = J
    S = vk.Solver([vk.upload_level(Lv, DEV) for Lv in P.levels])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vk_set_setup_variant(variant)
    with pytest.raises(vk.VkError) as e:
        S.vanka_setup(0.7)
    assert e.value.status == vk.VK_ERR_SINGULAR
    assert e.value.bad_level == 1 and e.value.bad_cell == cell
    S.close()


def test_singular_coarser_patch_reported_by_the_solve(vk):
    """A zero pivot in a patch below the finest level.  The coarser levels' inversions run on beside
    the next solve, so vanka_setup returns and the solve names the level and cell (vanka_setup does
    where the library has no separate setup stream); setup must then run again."""
    P = build_problem("channel2d_44x8_k1", shape=(8, 4), levels=3)
    L = P.levels[1]
    assert L.mesh.n_K == 42 and P.levels[2].mesh.n_cells > L.mesh.n_cells
    cell = 5
    pdof = int(L.cell_dofs[cell][18])   # a pressure DoF: it belongs to this cell only
    J = L.J.tolil()
    J[pdof, :] = 0.0
    J = J.tocsr()
    J.eliminate_zeros()
    J.sort_indices()
    L.J = J
    S = vk.Solver([vk.upload_level(Lv, DEV) for Lv in P.levels])
    S.vk_set_workspace("f64", 30, device=DEV)
    b = torch.from_numpy(P.b).to(DEV)
    x = torch.zeros_like(b)
    try:
        S.vanka_setup(0.7)
    except vk.VkError as e:
        assert e.status == vk.VK_ERR_SINGULAR and e.bad_level == 1 and e.bad_cell == cell
        S.close()
        return
    with pytest.raises(vk.VkError) as e:
        S.gmres_solve(b, x, rtol=1e-8)
    assert e.value.status == vk.VK_ERR_SINGULAR
    assert f"cell {cell} on level 1" in str(e.value)
    with pytest.raises(vk.VkError) as e2:
        S.vcycle(b, x, 2, 2)
    assert e2.value.status == vk.VK_ERR_STATE
    # the same through a direct entry point: vanka_smooth on the finest level reads the status
    S.vanka_setup(0.7)
    with pytest.raises(vk.VkError) as e3:
        S.vanka_smooth(2, b, x, 1, d_is_zero=True)
    assert e3.value.status == vk.VK_ERR_SINGULAR and f"cell {cell} on level 1" in str(e3.value)
    S.close()


def test_malformed_csr_rejected(vk):
    P = build_problem("channel2d_44x8_k1", shape=(8, 4), levels=2)
    lv = [vk.upload_level(L, DEV) for L in P.levels]
    col = lv[1]["J"]["col"].clone()
    col[3], col[4] = lv[1]["J"]["col"][4], lv[1]["J"]["col"][3]     # unsorted row
    bad = dict(lv[1])
    bad["J"] = dict(lv[1]["J"], col=col)
    with pytest.raises(vk.VkError) as e:
        vk.Solver([lv[0], bad])
    assert e.value.status == vk.VK_ERR_ARG
    col2 = lv[1]["J"]["col"].clone()
    col2[7] = P.finest.n + 5                                           # out of range
    bad["J"] = dict(lv[1]["J"], col=col2)
    with pytest.raises(vk.VkError) as e:
        vk.Solver([lv[0], bad])
    assert e.value.status == vk.VK_ERR_ARG
    cd = lv[1]["cell_dofs"].clone()
    cd[0, 0] = -1
    bad = dict(lv[1], cell_dofs=cd)
    with pytest.raises(vk.VkError) as e:
        vk.Solver([lv[0], bad])
    assert e.value.status == vk.VK_ERR_ARG


def test_timing_counts(vk):
    P, _ = problem("cfg0")
    S = make_solver(vk, P)
    S.vk_timing_enable(True)
    L = P.finest
    d = torch.zeros(L.n, dtype=torch.float64, device=DEV)
    S.vanka_smooth(len(P.levels) - 1, t(P.b), d, 3, d_is_zero=True)
    n, ms = S.vk_timing_read("patch_gemv", len(P.levels) - 1)
    assert n == 3 and ms > 0
    n, ms = S.vk_timing_read("dof_gather", len(P.levels) - 1)
    assert n == 3 and ms > 0
    n, ms = S.vk_timing_read("spmv", len(P.levels) - 1)
    assert n == 2
    S.vk_timing_enable(False)


def test_timing_kinds_and_sampling(vk):
    """vk_timing_kinds records only the chosen classes, one launch in `every` (counting from the
    first), and timing does not change the result."""
    P, _ = problem("cfg0")
    S = make_solver(vk, P)
    l = len(P.levels) - 1
    L = P.finest
    d = torch.zeros(L.n, dtype=torch.float64, device=DEV)
    S.vanka_smooth(l, t(P.b), d, 7, d_is_zero=True)
    ref = d.cpu().numpy()
    for every, expect in ((1, 7), (3, 3), (7, 1)):
        S.vk_timing_kinds(["patch_gemv"], every)
        S.vk_timing_enable(True, l)
        d.zero_()
        S.vanka_smooth(l, t(P.b), d, 7, d_is_zero=True)
        n, ms = S.vk_timing_read("patch_gemv", l)
        assert n == expect and ms > 0, (every, n)
        assert S.vk_timing_read("spmv", l)[0] == 0 and S.vk_timing_read("dof_gather", l)[0] == 0
        S.vk_timing_enable(False)
        np.testing.assert_array_equal(d.cpu().numpy(), ref)
    with pytest.raises(vk.VkError) as e:
        S.vk_timing_kinds(["patch_gemv"], 0)
    assert e.value.status == vk.VK_ERR_ARG
    S.vk_timing_kinds(None)
    S.close()


@pytest.mark.parametrize("tile", [1, 2, 4, 8])
def test_patch_tiles_agree(vk, tile):
    P, H = problem("ragged_k2")
    S = make_solver(vk, P)
    l = len(P.levels) - 1
    try:
        S.vk_set_patch_tile(l, tile)
    except vk.VkError:
        pytest.skip("tile too narrow for this patch")
    rng = np.random.default_rng(6)
    b = rng.standard_normal(P.finest.n)
    d0 = rng.standard_normal(P.finest.n)
    d = t(d0)
    S.vanka_smooth(l, t(b), d, 1)
    assert rel(d.cpu().numpy(), H.smooth(l, b, d0, 1)) <= 1e-10


@pytest.mark.parametrize("variant", ["dof_gather", "coloured_scatter", "dof_gather_offsets"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sweep_variants(vk, variant, prec):
    """Both implementations of the averaged additive sweep equal the oracle's Eq. 3.5."""
    P, H = problem("ragged_k2")
    S = make_solver(vk, P, prec=prec)
    S.vk_set_sweep_variant(variant)
    Href = H if prec == "f64" else oracle.OracleHierarchy(P.levels, patch_store=oracle.round_f32)
    tol = 1e-10 if prec == "f64" else 2e-5
    rng = np.random.default_rng(7)
    for l in range(1, len(P.levels)):
        L = P.levels[l]
        b = rng.standard_normal(L.n)
        d0 = rng.standard_normal(L.n)
        d = t(d0)
        S.vanka_smooth(l, t(b), d, 2)
        assert rel(d.cpu().numpy(), Href.smooth(l, b, d0, 2)) <= tol


@pytest.mark.parametrize("case", ["cfg0", "box3d"])
def test_dof_gather_widths_agree(vk, case):
    """The fixed-width and the offset-list DoF gathers give the same sweep bit for bit (the same
    sums in the same order); cfg0 has 4-wide lists (2D), the box 8-wide (3D)."""
    P, _ = problem(case)
    outs = []
    for variant in ("dof_gather", "dof_gather_offsets"):
        S = make_solver(vk, P, prec="f32")
        S.vk_set_sweep_variant(variant)
        rng = np.random.default_rng(8)
        l = len(P.levels) - 1
        b = rng.standard_normal(P.finest.n)
        d = t(rng.standard_normal(P.finest.n))
        S.vanka_smooth(l, t(b), d, 2)
        outs.append(d.cpu().numpy())
        S.close()
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("case", ["cfg0", "ragged_k2", "k3", "box3d", "k4", "box3d_k0", "r4_k1", "r4_k2",
                                  "box3d_k2", "r4_k3"])
def test_setup_variants_agree(vk, case):
    """The register-resident (or, for the widest patches, the blocked) and the LDS / global-memory
    Gauss-Jordan kernels give the same inverses (variant 3: the matrix-core kernel gathering through
    the LDS hash instead of the patch entry map)."""
    P, H = problem(case)
    outs = []
    for variant in (0, 1, 2, 3):
        S = vk.Solver([vk.upload_level(L, DEV) for L in P.levels])
        S.vk_set_workspace("f64", 30, device=DEV)
        S.vk_set_setup_variant(variant)
        S.vanka_setup(0.7)
        l = len(P.levels) - 1
        nc, nK = P.finest.mesh.n_cells, P.finest.mesh.n_K
        out = torch.empty((nc, nK, nK), dtype=torch.float64, device=DEV)
        S.vk_get_patch_inverses(l, 0, nc, out)
        outs.append(out.cpu().numpy())
        err = np.abs(outs[-1] - H.A[l]).max(axis=(1, 2)) / np.abs(H.A[l]).max(axis=(1, 2))
        assert err.max() <= 1e-10, (variant, err.max())


def test_coarse_inverse_cfg1_size(vk):
    """The blocked coarse inverse at the 11x2 dG(2) coarse level (888 unknowns, several panels)."""
    P = build_problem("channel2d_176x32_k2", shape=(22, 4), levels=2)
    S = make_solver(vk, P)
    J0 = P.levels[0].J.toarray()
    n0 = J0.shape[0]
    out = torch.empty((n0, n0), dtype=torch.float64, device=DEV)
    S.vk_get_coarse_inverse(out)
    ref = np.linalg.inv(J0)
    kappa = np.linalg.cond(J0)
    assert rel(out.cpu().numpy(), ref) <= 100 * kappa * np.finfo(float).eps


def test_autotuned_matches_oracle(vk):
    """Tuned launch shapes change only the summation order."""
    P, H = problem("cfg0")
    S = make_solver(vk, P)
    S.vk_autotune(3)
    S.vanka_setup(0.7)
    b = np.random.default_rng(8).standard_normal(P.finest.n)
    x = torch.empty(P.finest.n, dtype=torch.float64, device=DEV)
    S.vcycle(t(b), x, 2, 2)
    assert rel(x.cpu().numpy(), oracle.vcycle(H, b, 2, 2)) <= 1e-10


@pytest.mark.parametrize("solver, pivoting", [(0, 0), (1, 0), (1, 1)])
def test_coarse_solve_3d_box_size(vk, solver, pivoting):
    """The 3D box's coarsest level (25 x 2 x 2 hexahedra, dG(1), n = 8 450, the largest directly
    solved block) on its own: the one-level V-cycle is the direct solve; it agrees with a sparse
    LU solve and leaves a residual at rounding level, through the block-tridiagonal factorisation
    (solver 0: level-set blocks) and through the dense inverse with the pivots chosen by tournament
    (pivoting 0) and by partial pivoting over all rows (1)."""
    import time
    import scipy.sparse.linalg as spla
    from synth.assemble import assemble_jacobian
    from synth.mesh import StructuredMesh
    from synth.problems import Level, inflow_state
    m = StructuredMesh((25, 2, 2), (2.5, 0.41, 0.41), 1)
    V = inflow_state(m, 0.45, np.random.default_rng(1002))
    J = assemble_jacobian(m, V, 1e-3, 0.01)
    assert J.shape[0] == 8450
    lv = Level(mesh=m, J=J, P=None, R=None, cell_dofs=m.cell_dofs(), colours=m.colours(), state=V)
    S = vk.Solver([vk.upload_level(lv, DEV)])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vk_set_coarse_solver(solver)
    S.vk_set_coarse_pivoting(pivoting)
    _say(f"coarse 8450 setup, solver {solver}, pivoting {pivoting}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.vanka_setup(0.7, "additive")
    torch.cuda.synchronize()
    _say(f"coarse 8450 setup {1e3 * (time.perf_counter() - t0):.1f} ms")
    nb, flops = S.vk_coarse_plan(0)
    if solver == 0:
        assert nb >= 3 and flops < 2.0 * 8450.0 ** 3 / 10  # level-set blocks, a fraction of the dense flops
    else:
        assert nb == 0 and flops == 2.0 * 8450.0 ** 3
    b = np.random.default_rng(7).standard_normal(J.shape[0])
    x = torch.empty(J.shape[0], dtype=torch.float64, device=DEV)
    S.vcycle(t(b), x, 0, 0)
    xg = x.cpu().numpy()
    xs = spla.spsolve(J.tocsc(), b)
    assert np.linalg.norm(xg - xs) <= 1e-9 * np.linalg.norm(xs)
    assert np.linalg.norm(J @ xg - b) <= 1e-11 * np.linalg.norm(b) * max(1.0, abs(J).max())
    S.close()


@pytest.mark.parametrize("pivoting", [0, 2])
@pytest.mark.parametrize("n", [64, 256, 1024, 2048, 4096])
def test_coarse_inverse_with_tied_pivots(vk, n, pivoting):
    """A Hadamard matrix (all entries +-1: every column's candidates tie in |a| at the first step,
    and ties recur) through the blocked Gauss-Jordan path of each block size, with the default pivot
    choice and with the tournament (2): its inverse is H^T / n.  Sizes cover one panel width and several
    outer blocks (64 columns each) per block kernel shape."""
    import types
    import scipy.linalg
    import scipy.sparse as sp
    H = scipy.linalg.hadamard(n).astype(np.float64)
    lv = types.SimpleNamespace(J=sp.csr_matrix(H), P=None, R=None, cell_dofs=np.zeros((1, 1), np.int32),
                               colours=np.zeros(1, np.int32))
    S = vk.Solver([vk.upload_level(lv, DEV)])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vk_set_coarse_pivoting(pivoting)
    S.vanka_setup(0.7, "additive")
    out = torch.empty((n, n), dtype=torch.float64, device=DEV)
    S.vk_get_coarse_inverse(out)
    # H is orthogonal up to the factor n (condition number 1): a wrong or inconsistent pivot choice
    # shows as an O(1) error or a singular-block report, rounding stays far below this bound
    assert rel(out.cpu().numpy(), H.T / n) <= 1e-10
    S.close()


def _channel_coarse_level(shape=(44, 8), singular_row=None):
    """One level of the 2D channel (k = 1) as a directly solved block: n = 8 164 on 44 x 8 cells."""
    from synth.assemble import assemble_jacobian
    from synth.mesh import StructuredMesh
    from synth.problems import Level, inflow_state, H_CHANNEL
    m = StructuredMesh(shape, (2.2, H_CHANNEL), 1)
    V = inflow_state(m, 0.3, np.random.default_rng(1003))
    J = assemble_jacobian(m, V, 1e-3, 0.01).tocsr()
    if singular_row is not None:
        J.data[J.indptr[singular_row]:J.indptr[singular_row + 1]] = 0.0
    return Level(mesh=m, J=J, P=None, R=None, cell_dofs=m.cell_dofs(), colours=m.colours(), state=V)


@pytest.mark.parametrize("solver", [0, 1])
def test_block_tridiagonal_coarse_solve_2d(vk, solver):
    """The 44 x 8 channel (n = 8 164) as the coarsest level: its level sets along the channel make a
    block-tridiagonal factorisation (solver 0); the direct solve agrees with a sparse LU solve and
    with the dense inverse's solve (solver 1) to rounding."""
    import scipy.sparse.linalg as spla
    lv = _channel_coarse_level()
    J = lv.J
    S = vk.Solver([vk.upload_level(lv, DEV)])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vk_set_coarse_solver(solver)
    S.vanka_setup(0.7, "additive")
    nb, _ = S.vk_coarse_plan(0)
    assert (nb >= 3) if solver == 0 else (nb == 0)
    b = np.random.default_rng(11).standard_normal(J.shape[0])
    x = torch.empty(J.shape[0], dtype=torch.float64, device=DEV)
    for rep in range(2):  # a second setup and solve reuse the plan
        S.vcycle(t(b), x, 0, 0)
        xs = spla.spsolve(J.tocsc(), b)
        assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs), rep
        S.vanka_setup(0.7, "additive")
    if solver == 0:
        with pytest.raises(vk.VkError, match="factorised"):
            S.vk_get_coarse_inverse(torch.empty((J.shape[0], J.shape[0]), dtype=torch.float64, device=DEV))
    S.close()


def test_block_tridiagonal_singular_reported(vk):
    """A zero row in the 44 x 8 channel's matrix: a Schur-complement block of the factorisation has no
    nonzero pivot left, and the first solve reports the coarse block as singular."""
    lv = _channel_coarse_level(singular_row=1234)
    S = vk.Solver([vk.upload_level(lv, DEV)])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vanka_setup(0.7, "additive")
    assert S.vk_coarse_plan(0)[0] >= 3
    b = t(np.ones(lv.J.shape[0]))
    x = torch.zeros_like(b)
    with pytest.raises(vk.VkError, match="singular"):
        S.vcycle(b, x, 0, 0)
    S.close()


def test_coarse_solver_mode_rejected(vk):
    P, _ = problem("cfg0")
    S = make_solver(vk, P)
    with pytest.raises(vk.VkError, match="coarse solver"):
        S.vk_set_coarse_solver(2)
    S.close()


def _dense_level(A):
    import types
    import scipy.sparse as sp
    return types.SimpleNamespace(J=sp.csr_matrix(A), P=None, R=None, cell_dofs=np.zeros((1, 1), np.int32),
                                 colours=np.zeros(1, np.int32))


def _saddle(n, m, seed):
    """[[K, B^T], [B, 0]] with K symmetric positive definite and B of full rank: the zero block
    makes pivoting across distant rows necessary (no pressure row can pivot its own column)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    K = G @ G.T / n + np.eye(n)
    B = rng.standard_normal((m, n))
    A = np.zeros((n + m, n + m))
    A[:n, :n] = K
    A[:n, n:] = B.T
    A[n:, :n] = B
    perm = rng.permutation(n + m)  # interleave the two kinds of rows
    return A[np.ix_(perm, perm)]


@pytest.mark.parametrize("n, kind", [(2049, "gauss"), (3001, "gauss"), (2600, "saddle"), (4100, "saddle")])
def test_wide_coarse_inverse_pivoting_modes(vk, n, kind):
    """Dense blocks of 2 049 to 4 100 rows (ragged against the 16-column panels, the 64-column tiles
    and the 512-row leaves): the inverse with the default pivot choice (0: the tournament above 4 096
    rows), partial pivoting over all rows (1) and the tournament (2) all match numpy's inverse, within
    1e4 eps times the condition number, and agree with each other."""
    if kind == "gauss":
        A = np.random.default_rng(n).standard_normal((n, n))
    else:
        A = _saddle(n - n // 5, n // 5, n)
    ref = np.linalg.inv(A)
    cond = np.linalg.cond(A)
    outs = []
    for mode in (0, 1, 2):
        S = vk.Solver([vk.upload_level(_dense_level(A), DEV)])
        S.vk_set_workspace("f64", 30, device=DEV)
        S.vk_set_coarse_pivoting(mode)
        S.vanka_setup(0.7, "additive")
        out = torch.empty((n, n), dtype=torch.float64, device=DEV)
        S.vk_get_coarse_inverse(out)
        outs.append(out.cpu().numpy())
        S.close()
        # a wrong pivot or a skipped step shows as an O(1) error; rounding stays within eps cond
        assert rel(outs[-1], ref) <= 1e4 * 2.2e-16 * cond, (mode, rel(outs[-1], ref), cond)
    assert rel(outs[2], outs[1]) <= 1e4 * 2.2e-16 * cond
    assert rel(outs[0], outs[2 if n > 4096 else 1]) == 0.0  # the default picks one of the two


@pytest.mark.parametrize("pivoting", [1, 2])
@pytest.mark.parametrize("defect", ["column", "row"])
def test_singular_wide_coarse_block_reported(vk, pivoting, defect):
    """A 3 000-row block with a zero column (or row), which the elimination keeps exactly zero: no
    nonzero pivot is left for that column (for the last column), so the first solve reports the block
    as singular under both pivot choices."""
    n = 3000
    A = np.random.default_rng(5).standard_normal((n, n))
    if defect == "column":
        A[:, 2500] = 0.0
    else:
        A[1234, :] = 0.0
    S = vk.Solver([vk.upload_level(_dense_level(A), DEV)])
    S.vk_set_workspace("f64", 30, device=DEV)
    S.vk_set_coarse_pivoting(pivoting)
    S.vanka_setup(0.7, "additive")
    b = t(np.ones(n))
    x = torch.zeros_like(b)
    with pytest.raises(vk.VkError, match="singular"):
        S.vcycle(b, x, 0, 0)
    S.close()


def test_coarse_pivoting_mode_rejected(vk):
    P, _ = problem("cfg0")
    S = make_solver(vk, P)
    with pytest.raises(vk.VkError, match="pivoting"):
        S.vk_set_coarse_pivoting(3)
    S.close()


def test_singular_coarse_block_reported_by_the_solve(vk):
    """The block inversion overlaps the next solve: a singular coarse matrix is reported by the first
    call that applies it, and setup must run again before the next solve."""
    import copy
    P, _ = problem("cfg0")
    levels = copy.copy(P.levels)
    L0 = copy.copy(levels[0])
    J0 = L0.J.copy()
    J0.data[J0.indptr[5]:J0.indptr[6]] = 0.0   # a zero row: J_0 is singular
    L0.J = J0
    levels[0] = L0
    for call in ("gmres", "vcycle"):
        S = make_solver(vk, type("P", (), {"levels": levels})())
        b = t(P.b)
        x = torch.zeros_like(b)
        with pytest.raises(vk.VkError, match="singular"):
            if call == "gmres":
                S.gmres_solve(b, x)
            else:
                S.vcycle(b, x, 2, 2)
        with pytest.raises(vk.VkError, match="vanka_setup"):
            S.gmres_solve(b, x)
        S.close()


def test_colouring_conflict_rejected(vk):
    """Cells of one colour must share no DoF (the coloured scatter and the multiplicative sweep
    update concurrently within a colour): a colouring that puts neighbours together is refused."""
    P, _ = problem("cfg0")
    ups = [vk.upload_level(L, DEV) for L in P.levels]
    lv = ups[-1]
    n = int(lv["n_cells"])
    lv["colour_cells"] = torch.arange(n, dtype=torch.int32, device=DEV)
    lv["colour_ptr"] = np.array([0, n], dtype=np.int32)
    lv["n_colours"] = 1
    S = vk.Solver(ups)
    S.vk_set_workspace("f64", 30, device=DEV)
    with pytest.raises(vk.VkError) as e:
        S.vanka_setup(0.7, "additive")
    assert e.value.status == vk.VK_ERR_ARG and "colour" in str(e.value)
    S.close()


@pytest.mark.parametrize("restart,max_iter", [(3, 200), (30, 5), (4, 6)])
def test_gmres_lookahead_restarts_and_limits(vk, restart, max_iter):
    """Several Arnoldi steps are enqueued between looks at the residual estimates; steps past the
    stopping step must not change the iterate, across restarts and at the iteration limit."""
    P, H = problem("cfg0")
    S = make_solver(vk, P)
    b = P.b
    x = torch.zeros(P.finest.n, dtype=torch.float64, device=DEV)
    its, relres, hist, ok = S.gmres_solve(t(b), x, restart=restart, max_iter=max_iter, rtol=1e-8,
                                          raise_on_noconv=False)
    xo, its_o, hist_o, ok_o, rel_o = oracle.gmres(P.finest.J, b, lambda v: oracle.vcycle(H, v, 2, 2),
                                                  restart=restart, max_iter=max_iter)
    xg = x.cpu().numpy()
    true_rel = np.linalg.norm(b - P.finest.J @ xg) / np.linalg.norm(b)
    _say(f"restart {restart} max_iter {max_iter}: {its} its (oracle {its_o}), ok {ok}")
    assert ok == ok_o
    assert abs(true_rel - relres) <= 1e-12
    if ok:
        assert abs(its - its_o) <= 1 and true_rel <= 1e-8
    else:
        assert its == max_iter == its_o
        assert rel(xg, xo) <= 1e-6
    k = min(len(hist), len(hist_o))
    np.testing.assert_allclose(hist[:k], hist_o[:k], rtol=1e-6)
