"""hipGraph replay of the V-cycle and of the Arnoldi steps.

Every replay must equal the eager launches bit for bit (the same kernels run with
the same arguments in the same order).  Each test replays several times with
eager work and synchronisations in between and checks every replay, and checks
that a change of a baked-in parameter (omega, tile, sweep variant) makes the
next call record a new graph whose result equals the eager result under the new
parameter.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import build_problem  # noqa: E402
from synth.batch import build_batch  # noqa: E402

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


@pytest.fixture(scope="module")
def cfg0():
    return build_problem("channel2d_44x8_k1")


def solver(vk, P, prec="f64"):
    S = vk.Solver([vk.upload_level(L, DEV) for L in P.levels])
    S.vk_set_workspace(prec, 30, device=DEV)
    S.vanka_setup(0.7, "additive")
    return S


def eager_noise():
    """Unrelated eager work on the current stream between replays."""
    a = torch.randn(1 << 16, device=DEV, dtype=torch.float64)
    (a * 2.0 + 1.0).sum().item()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_gmres_replays_equal_eager(vk, cfg0, prec):
    P = cfg0
    S = solver(vk, P, prec)
    b = torch.from_numpy(P.b).to(DEV)
    x = torch.zeros_like(b)
    _say(f"graph gmres eager {prec}")
    its_e, rel_e, hist_e, ok = S.gmres_solve(b, x, restart=30, max_iter=200, rtol=1e-8)
    assert ok
    xe = x.cpu().numpy()
    S.vk_set_graphs(True)
    for rep in range(4):
        _say(f"graph gmres replay {rep}")
        # a new setup with unchanged omega refills the inverses in place: no new recording
        S.vanka_setup(0.7, "additive")
        x.zero_()
        its, rel, hist, ok = S.gmres_solve(b, x, restart=30, max_iter=200, rtol=1e-8)
        torch.cuda.synchronize()
        assert ok and its == its_e and rel == rel_e
        np.testing.assert_array_equal(hist, hist_e)
        np.testing.assert_array_equal(x.cpu().numpy(), xe)
        eager_noise()
    # after each setup the first Arnoldi step runs eagerly (it overlaps the coarse inversion)
    captures, launches = S.vk_graph_stats()
    assert captures == its_e - 1 and launches == 4 * (its_e - 1), (captures, launches, its_e)
    S.close()


def test_graph_vcycle_recaptures_on_change(vk, cfg0):
    P = cfg0
    S = solver(vk, P)
    b = torch.from_numpy(P.b).to(DEV)
    x = torch.empty_like(b)

    def eager(setup):
        S.vk_set_graphs(False)
        setup()
        S.vcycle(b, x, 2, 2)
        torch.cuda.synchronize()
        return x.cpu().numpy()

    changes = [
        ("omega 0.7", lambda: S.vanka_setup(0.7, "additive")),
        ("omega 0.5", lambda: S.vanka_setup(0.5, "additive")),
        ("tile 2", lambda: S.vk_set_patch_tile(len(P.levels) - 1, 2)),
        ("coloured scatter", lambda: S.vk_set_sweep_variant("coloured_scatter")),
        ("nu (1, 3)", None),
    ]
    prev_captures = 0
    for name, change in changes:
        nu = (1, 3) if change is None else (2, 2)
        _say(f"graph vcycle {name}")
        if change is None:
            S.vk_set_graphs(False)
            S.vcycle(b, x, *nu)
            torch.cuda.synchronize()
            ref = x.cpu().numpy()
        else:
            ref = eager(change)
        S.vk_set_graphs(True)
        for rep in range(3):
            x.fill_(float("nan"))
            S.vcycle(b, x, *nu)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(x.cpu().numpy(), ref, err_msg=f"{name} replay {rep}")
            eager_noise()
        captures, _ = S.vk_graph_stats()
        assert captures == prev_captures + 1, (name, captures)
        prev_captures = captures
    S.close()


def test_graph_batched_gmres_replays_equal_eager(vk):
    B = build_batch(n_systems=5, seed=2, nx8=(1, 3), ny8=(1, 2), max_coarse_unknowns=300)
    S = vk.Solver([vk.upload_packed_level(L, DEV) for L in B.levels])
    S.vk_set_segments(B.seg_rows)
    S.vk_set_workspace("f32", 30, device=DEV)
    S.vanka_setup(0.7)
    b = torch.from_numpy(B.b).to(DEV)
    x = torch.zeros_like(b)
    _say("graph batched eager")
    its_e, rel_e, conv = S.gmres_solve_batched(b, x, restart=30, max_iter=200, rtol=1e-8)
    assert conv
    xe = x.cpu().numpy()
    S.vk_set_graphs(True)
    for rep in range(3):
        _say(f"graph batched replay {rep}")
        x.zero_()
        its, rel, conv = S.gmres_solve_batched(b, x, restart=30, max_iter=200, rtol=1e-8)
        torch.cuda.synchronize()
        assert conv
        np.testing.assert_array_equal(its, its_e)
        np.testing.assert_array_equal(rel, rel_e)
        np.testing.assert_array_equal(x.cpu().numpy(), xe)
        eager_noise()
    captures, launches = S.vk_graph_stats()
    assert captures == its_e.max() and launches == 3 * its_e.max()
    S.close()


def test_graph_timing_runs_eager(vk, cfg0):
    """With event timing on, steps are launched eagerly (no recording)."""
    P = cfg0
    S = solver(vk, P)
    S.vk_set_graphs(True)
    S.vk_timing_enable(True, len(P.levels) - 1)
    b = torch.from_numpy(P.b).to(DEV)
    x = torch.zeros_like(b)
    its, *_ = S.gmres_solve(b, x)
    n_gemv, _ = S.vk_timing_read("patch_gemv", len(P.levels) - 1)
    S.vk_timing_enable(False)
    assert S.vk_graph_stats() == (0, 0)
    assert n_gemv == 4 * its
    S.close()
