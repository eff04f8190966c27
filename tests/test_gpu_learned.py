"""Learned initial guess on the GPU: the BF16 network kernels against the FP64
oracle, the patch kernels against their definitions, the Newton march against
the oracle's, and the trained network's gain over the extrapolation.

Tolerances (normwise relative):
  * forward output against the oracle with the same BF16 rounding points: 5e-3
    (FP32 accumulation order, tanhf, and the rare BF16 rounding decision that
    flips with it: one unit roundoff 2^-9 on a few entries);
  * against the unrounded FP64 network: 5e-2 (three roundings of relative
    2^-9 per layer over four layers, as in the oracle's own bound);
  * gradients: 2e-2 with the same rounding points, 8e-2 unrounded (the
    backward pass adds a BF16 rounding of every pre-activation gradient);
  * Adam: 1e-5 (FP32 arithmetic against FP64).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import mlp as omlp  # noqa: E402
from oracle.precision import round_bf16  # noqa: E402
from synth.learned import init_mlp_params, minibatch_orders, mlp_layer_shapes  # noqa: E402
from synth.march import ChannelMarch  # noqa: E402

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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def bf16_tensor(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(DEV)


def net_case(seed, n_in=84, width=128, n_hidden=3, n_out=42, n_rows=400):
    shapes = mlp_layer_shapes(n_in, width, n_hidden, n_out)
    p = init_mlp_params(n_in, width, n_hidden, n_out, seed=seed)
    rng = np.random.default_rng(200 + seed)
    p = (p + 0.02 * rng.standard_normal(p.size)).astype(np.float32)
    Xf = round_bf16(rng.standard_normal((n_rows, n_in)))
    T = rng.standard_normal((n_rows, n_out)).astype(np.float32)
    return shapes, p, Xf, T


@pytest.mark.parametrize("batch,indexed", [(173, True), (64, False), (1, True)])
def test_forward_matches_oracle(vk, batch, indexed):
    shapes, p, Xf, _ = net_case(1)
    net = vk.MLP(84, 128, 3, 42, 512, device=DEV)
    net.set_params(torch.from_numpy(p).to(DEV))
    rows = np.random.default_rng(3).permutation(Xf.shape[0])[:batch].astype(np.int32) if indexed else None
    _say(f"mlp forward batch {batch} indexed {indexed}")
    if indexed:
        y = net.forward(bf16_tensor(Xf), rows=torch.from_numpy(rows).to(DEV))
    else:
        y = net.forward(bf16_tensor(Xf[:batch]))
    y = y.cpu().numpy().astype(np.float64)
    Xb = Xf[rows] if indexed else Xf[:batch]
    _, y_r = omlp.forward(p.astype(np.float64), shapes, Xb, bf16_points=True)
    _, y_64 = omlp.forward(p.astype(np.float64), shapes, Xb)
    assert rel(y, y_r) <= 5e-3, rel(y, y_r)
    assert rel(y, y_64) <= 5e-2, rel(y, y_64)


def test_gemm_lane_layout_small_shapes(vk):
    """Single-layer networks of odd sizes: checks the matrix-core operand layout on ragged tiles."""
    for (n_in, n_out, batch) in [(3, 5, 7), (17, 33, 19), (40, 1, 31)]:
        shapes = mlp_layer_shapes(n_in, 16, 1, n_out)
        rng = np.random.default_rng(n_in)
        p = rng.standard_normal(omlp.n_params(shapes)).astype(np.float32) * 0.3
        Xf = round_bf16(rng.standard_normal((batch, n_in)))
        net = vk.MLP(n_in, 16, 1, n_out, 64, device=DEV)
        net.set_params(torch.from_numpy(p).to(DEV))
        y = net.forward(bf16_tensor(Xf)).cpu().numpy()
        _, y_r = omlp.forward(p.astype(np.float64), shapes, Xf, bf16_points=True)
        assert rel(y, y_r) <= 5e-3, (n_in, n_out, batch, rel(y, y_r))


@pytest.mark.parametrize("batch", [300, 16])
def test_gradient_matches_oracle(vk, batch):
    shapes, p, Xf, T = net_case(2)
    net = vk.MLP(84, 128, 3, 42, 512, device=DEV)
    net.set_params(torch.from_numpy(p).to(DEV))
    rows = np.random.default_rng(5).permutation(Xf.shape[0])[:batch].astype(np.int32)
    _say(f"mlp gradient batch {batch}")
    loss, g = net.gradient(bf16_tensor(Xf), torch.from_numpy(T).to(DEV), rows=torch.from_numpy(rows).to(DEV))
    g = g.cpu().numpy().astype(np.float64)
    L_r, g_r = omlp.loss_and_grad(p.astype(np.float64), shapes, Xf[rows], T[rows].astype(np.float64),
                                  bf16_points=True)
    L_64, g_64 = omlp.loss_and_grad(p.astype(np.float64), shapes, Xf[rows], T[rows].astype(np.float64))
    assert abs(float(loss.item()) - L_r) <= 5e-3 * L_r
    off = 0
    for (o, i) in shapes:
        for size in (o * i, o):
            sl = slice(off, off + size)
            assert rel(g[sl], g_r[sl]) <= 2e-2, (o, i, size, rel(g[sl], g_r[sl]))
            off += size
    assert rel(g, g_64) <= 8e-2, rel(g, g_64)


def test_adam_matches_oracle(vk):
    shapes, p, Xf, T = net_case(3)
    net = vk.MLP(84, 128, 3, 42, 512, device=DEV)
    net.set_params(torch.from_numpy(p).to(DEV))
    x, t = bf16_tensor(Xf), torch.from_numpy(T).to(DEV)
    th = p.astype(np.float64)
    m = v = np.zeros_like(th)
    for step in range(1, 4):
        _, g = net.gradient(x[:128], t[:128])
        net.adam(1e-3, 0.9, 0.999, 1e-8)
        th, m, v = omlp.adam_step(th, m, v, g.cpu().numpy().astype(np.float64), step, 1e-3)
        got = net.get_params().cpu().numpy()
        assert rel(got, th) <= 1e-5, (step, rel(got, th))


def test_adam_without_gradient_is_a_state_error(vk):
    net = vk.MLP(4, 8, 1, 2, 16, device=DEV)
    net.set_params(torch.zeros(net.n_params, device=DEV))
    with pytest.raises(vk.VkError, match="no gradient"):
        net.adam(1e-3)


def test_patch_kernels_match_definitions(vk):
    pr = ChannelMarch(shape=(10, 4), levels=2, k=1)
    m = pr.fine.mesh
    rng = np.random.default_rng(9)
    X1, X2, X3 = (rng.standard_normal(m.n) for _ in range(3))
    cd = m.cell_dofs()
    nK = m.n_K
    mean = rng.standard_normal(2 * nK).astype(np.float32)
    inv = (0.5 + rng.random(2 * nK)).astype(np.float32)
    net = vk.MLP(2 * nK, 16, 1, nK, m.n_cells, device=DEV)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    feat = torch.empty((m.n_cells, 2 * nK), dtype=torch.bfloat16, device=DEV)
    net.patch_features(t(cd), t(X1), t(X2), t(X3), t(mean), t(inv), feat)
    ref = np.concatenate([(X2 - X1)[cd], (X2 - X3)[cd]], axis=1)
    ref = (ref - mean.astype(np.float64)).astype(np.float32) * inv          # FP32 product, then BF16
    got = feat.float().cpu().numpy()
    np.testing.assert_array_equal(got, round_bf16(ref).astype(np.float32))
    # targets
    tg = torch.empty((m.n_cells, nK), dtype=torch.float32, device=DEV)
    net.patch_targets(t(cd), t(X3), t(X1), t(mean[:nK]), t(inv[:nK]), tg)
    ref_t = (((X3 - X1)[cd] - mean[:nK].astype(np.float64)) * inv[:nK].astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(tg.cpu().numpy(), ref_t)
    # averaged corrections
    pred = rng.standard_normal((m.n_cells, nK)).astype(np.float32)
    sd = (0.5 + rng.random(nK)).astype(np.float32)
    ptr, lst = vk.dof_entries(cd, m.n)
    out = torch.empty(m.n, dtype=torch.float64, device=DEV)
    net.patch_average(t(ptr), t(lst), nK, t(pred), t(mean[:nK]), t(sd), t(X2), out)
    corr = pred.astype(np.float64) * sd.astype(np.float64) + mean[:nK].astype(np.float64)
    acc = np.zeros(m.n)
    cnt = np.zeros(m.n)
    np.add.at(acc, cd.ravel(), corr.ravel())
    np.add.at(cnt, cd.ravel(), 1.0)
    np.testing.assert_allclose(out.cpu().numpy(), X2 + acc / cnt, rtol=1e-13, atol=1e-13)
    # extrapolation kernel
    ext = torch.empty(m.n, dtype=torch.float64, device=DEV)
    net.slab_extrapolate(pr.E, t(X1), ext)
    np.testing.assert_allclose(ext.cpu().numpy(), pr.extrapolate(X1), rtol=1e-15, atol=1e-15)


def test_newton_march_matches_oracle(vk):
    from paper_2210_02690_amd.guess import ExtrapolationGuess, NewtonMarch, march
    pr = ChannelMarch(shape=(8, 4), levels=2, k=1)
    nm = NewtonMarch(pr, device=DEV, prec="f64")
    slabs = [pr.initial_slab()]
    _say("newton march gpu")
    st = march(nm, 1, 3, slabs, ExtrapolationGuess(pr, DEV))
    Xs, counts = oracle.march(pr, 3)
    for n in range(1, 4):
        assert st[n - 1]["converged"] and st[n - 1]["newton"] == counts[n - 1][0]
        assert abs(st[n - 1]["gmres"] - counts[n - 1][1]) <= counts[n - 1][0]
        assert rel(slabs[n], Xs[n]) <= 1e-8, (n, rel(slabs[n], Xs[n]))
    nm.close()


def test_learned_guess_beats_extrapolation(vk):
    """Train on slabs 1..40 of a small channel whose inflow varies fast enough that Newton needs two
    steps per slab from the extrapolation (peak 1.0 (1 + 0.5 sin(2 pi t / 0.1)), ten slabs per
    period), evaluate slabs 41..56 three ways: extrapolation, the raw learned guess, and the judged
    guess (the one of the two with the smaller slab residual).  The judged guess never starts from a
    larger residual than the extrapolation and costs fewer Newton steps and GMRES iterations in
    total; all marches reach the same slab solutions.  The counts and times are printed."""
    from paper_2210_02690_amd.guess import ExtrapolationGuess, JudgedGuess, LearnedGuess, NewtonMarch, march
    pr = ChannelMarch(shape=(22, 4), levels=2, k=1, inflow=(1.0, 0.5, 0.1))
    nm = NewtonMarch(pr, device=DEV, prec="f32")
    slabs = [pr.initial_slab()]
    fb = ExtrapolationGuess(pr, DEV)
    _say("march 1..40")
    st0 = march(nm, 1, 40, slabs, fb)
    assert sum(s["newton"] for s in st0[5:]) >= 2 * len(st0[5:])  # the regime: >= 2 Newton steps per slab
    lg = LearnedGuess(pr, 128, 3, DEV)
    n_samples = (len(slabs) - 2) * pr.fine.mesh.n_cells
    params0 = init_mlp_params(2 * pr.fine.mesh.n_K, 128, 3, pr.fine.mesh.n_K, seed=0)
    _say("train")
    losses = lg.fit(slabs, params0, minibatch_orders(n_samples, 150, seed=0), batch=256, lr=2e-3)
    assert losses[-1] < 0.2 * losses[0], losses[::25]
    _say("evaluate")
    runs = {}
    for name, guess in (("extrapolation", fb), ("learned", lg), ("judged", JudgedGuess(lg, fb, pr))):
        run = list(slabs)
        st = march(nm, 41, 56, run, guess)
        runs[name] = (st, run)
        _say(f"{name}: newton {sum(s['newton'] for s in st)} {[s['newton'] for s in st]}, gmres "
             f"{sum(s['gmres'] for s in st)}, F0 mean {np.mean([s['F0'] for s in st]):.3e}, "
             f"solve {sum(s['t_solve'] for s in st):.2f} s")
    st_f, run_f = runs["extrapolation"]
    st_j, run_j = runs["judged"]
    assert all(s["converged"] for name in runs for s in runs[name][0])
    # the judge: never a larger starting residual than the fallback, never more Newton steps in total
    assert all(j["F0"] <= f["F0"] * (1 + 1e-12) for j, f in zip(st_j, st_f))
    assert sum(s["newton"] for s in st_j) <= sum(s["newton"] for s in st_f)
    # and in this regime the network pays: fewer Newton steps and fewer GMRES iterations in total
    # (measured 16 vs 32 and 112 vs 163)
    assert sum(s["newton"] for s in st_j) < sum(s["newton"] for s in st_f)
    assert sum(s["gmres"] for s in st_j) < sum(s["gmres"] for s in st_f)
    # every march reaches the same slab solutions (each solved to ||F|| < 1e-8)
    for name in ("learned", "judged"):
        assert rel(runs[name][1][-1], run_f[-1]) <= 1e-6, (name, rel(runs[name][1][-1], run_f[-1]))
    nm.close()
