"""Benchmark of the Vanka / multigrid / GMRES hot path on one MI355X.

One step = the whole hot path on one Newton system: vanka_setup (patch gather,
FP64 patch inverses stored in the chosen precision, coarse inverse) followed by
gmres_solve from x = 0 to a relative residual of 1e-8 (GMRES(30), one V-cycle
with 2 pre- and 2 post-smoothing additive coloured Vanka sweeps, omega = 0.7).
Default workload: the 100 x 16 x 16 hexahedral box, dG(1), Q2/P1disc (n_K = 170,
1 518 134 unknowns, 4 levels).

value = Vanka cell-sweeps performed per second over the timed steps: every
V-cycle applies nu_pre + nu_post sweeps on each level l >= 1, each sweep visits
every cell of the level once.  The headline runs with FP32 patch inverses; the
same line carries the FP64 leg, the GMRES time to 1e-8 of both, the roofline of
the whole finest-level sweep (with each of its kernels, the patch inversion and
the coarse block inversion beside it), the 176 x 32 dG(2) channel's figures and
the FP64 CPU oracle timed phase by phase on a bounded sample.

python bench.py [--steps K] [--warmup W] [--config NAME] [--prec f32|f64|bf16]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PREC_BYTES = {"f64": 8, "f32": 4, "bf16": 2}
# the timed region times one in TIMING_EVERY finest patch-GEMV launches (each recorded launch
# slows the stream by a few microseconds); 7 is prime to the launches per V-cycle, so the sample
# visits every sweep position (the first sweep of a V-cycle reads a colder defect than the rest)
TIMING_EVERY = 7


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cells_sweeps_per_vcycle(P, nu1, nu2):
    return sum(L.mesh.n_cells for L in P.levels[1:]) * (nu1 + nu2)


def patch_gemv_bytes(L, prec):
    """Algorithmic bytes of one patch-GEMV launch (all cells of level L):
    per cell the n_K^2 stored entries of A_K, the cell's DoF list (int32), the
    gathered defect entries (FP64) and the written products y_K (FP64 for FP64
    storage, FP32 otherwise)."""
    nK = L.mesh.n_K
    y_bytes = 8 if prec == "f64" else 4
    return L.mesh.n_cells * (nK * nK * PREC_BYTES[prec] + nK * (4 + 8 + y_bytes))


def run_step(S, b, x, nu, restart, max_iter):
    S.vanka_setup(0.7, "additive")
    x.zero_()
    its, rel, _, ok = S.gmres_solve(b, x, restart=restart, max_iter=max_iter, rtol=1e-8, nu_pre=nu[0],
                                    nu_post=nu[1])
    if not ok:
        raise RuntimeError(f"GMRES did not reach 1e-8 ({its} its, rel {rel:.2e})")
    return its, rel


def phase_times(torch, S, b, x, nu, restart, max_iter, reps=3):
    """Median setup and GMRES wall times (ms), each phase bracketed by syncs."""
    ts, tg = [], []
    its = rel = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.vanka_setup(0.7, "additive")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x.zero_()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        its, rel, _, ok = S.gmres_solve(b, x, restart=restart, max_iter=max_iter, rtol=1e-8,
                                        nu_pre=nu[0], nu_post=nu[1])
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ts.append((t1 - t0) * 1e3)
        tg.append((t3 - t2) * 1e3)
    return float(np.median(ts)), float(np.median(tg)), its, rel


def stream_rates_gbs(torch, dev, mib=1024, reps=5):
    """Rates (GB/s) of two plain torch kernels over a 1 GiB FP64 buffer on this GPU, beside the
    published peak: a device copy (read + written bytes) and a sum (read bytes; the patch GEMV
    reads 98 % of its bytes)."""
    n = (mib << 20) // 8
    src = torch.empty(n, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def rate(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return reps * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9

    copy = rate(lambda: dst.copy_(src), 2 * n * 8)
    read = rate(lambda: src.sum(), n * 8)
    del src, dst
    return copy, read


def sweep_rate(torch, S, P, b_np, sweeps=40):
    """Finest-level additive sweeps in isolation: cells*sweeps/s."""
    l = len(P.levels) - 1
    b = torch.from_numpy(b_np).cuda()
    d = torch.zeros_like(b)
    S.vanka_smooth(l, b, d, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.vanka_smooth(l, b, d, sweeps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return P.finest.mesh.n_cells * sweeps / dt


def timed_steps(torch, step, reps):
    """Wall time (s) of `reps` calls of step() bracketed by synchronisations, and their results."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(reps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res


def run_batch(args, torch, vk, dev):
    """64 independent systems (meshes 32x8 .. 128x24, k in {1,2,3}, seeded viscosities) in one
    context: one vanka_setup and one gmres_solve_batched per step.  value = useful cell-sweeps
    per second, summed over systems (each system's own iterations times its V-cycle's sweeps);
    the lockstep also sweeps systems that have already converged, counted separately."""
    from synth.batch import build_batch
    import oracle
    restart, max_iter, nu = 30, 300, (2, 2)
    t0 = time.perf_counter()
    B = build_batch(64, seed=0)
    fin = B.levels[-1]
    log(f"[bench] built batch: {len(B.systems)} systems, n = {fin.n}, finest cells = {B.n_cells_finest}, "
        f"{time.perf_counter() - t0:.1f} s")
    S = vk.Solver([vk.upload_packed_level(L, dev) for L in B.levels])
    S.vk_set_segments(B.seg_rows)
    S.vk_set_workspace(args.prec, restart, device=dev)
    S.vanka_setup(0.7, "additive")
    S.vk_autotune(10)
    b = torch.from_numpy(B.b).to(dev)
    x = torch.zeros_like(b)
    order = sorted(fin.rows.items(), key=lambda kv: kv[1][0])  # segment order
    cs_sys = np.array([sum(L.mesh.n_cells for L in B.hierarchies[si][1:]) * sum(nu) for si, _ in order])

    def step():
        S.vanka_setup(0.7, "additive")
        x.zero_()
        its, rel, conv = S.gmres_solve_batched(b, x, restart=restart, max_iter=max_iter, rtol=1e-8,
                                               nu_pre=nu[0], nu_post=nu[1])
        if not conv:
            raise RuntimeError("batched GMRES did not converge")
        return its, rel

    S.vk_set_graphs(not args.no_graphs)
    for w in range(args.warmup):
        its, rel = step()
        log(f"[bench] warmup {w}: its {its.min()}..{its.max()}")
    dt, res = timed_steps(torch, step, args.steps)
    its = res[-1][0]
    useful = sum(int((r[0] * cs_sys).sum()) for r in res)
    performed = sum(int(r[0].max()) * int(cs_sys.sum()) for r in res)
    value = useful / dt
    ms_per_step = dt / args.steps * 1e3
    log(f"[bench] batch timed {args.steps} steps in {dt:.3f} s")
    graph_stats = S.vk_graph_stats()

    # eager pass with event timing of the finest level: roofline of the patch GEMV (one launch
    # per patch width) and phase times
    S.vk_set_graphs(False)
    l_fine = len(B.levels) - 1
    S.vk_timing_kinds(["patch_gemv"])  # every launch: one per patch width, of different sizes
    S.vk_timing_enable(True, l_fine)
    dt_e, res_e = timed_steps(torch, step, max(3, args.steps // 4))
    n_apply, ms_apply = S.vk_timing_read("patch_gemv", l_fine)
    S.vk_timing_enable(False)
    S.vk_timing_kinds(None)
    bytes_sweep = sum(g["cell_dofs"].shape[0] * (g["n_K"] ** 2 * PREC_BYTES[args.prec]
                                                 + g["n_K"] * (4 + 8 + (8 if args.prec == "f64" else 4)))
                      for g in fin.groups)
    n_sweeps = n_apply / max(len(fin.groups), 1)
    achieved = bytes_sweep * n_sweeps / (ms_apply * 1e-3) / 1e9
    setup_ms = []
    gm_ms = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.vanka_setup(0.7, "additive")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x.zero_()
        S.vk_set_graphs(not args.no_graphs)
        S.gmres_solve_batched(b, x, restart=restart, max_iter=max_iter, rtol=1e-8, nu_pre=nu[0], nu_post=nu[1])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        setup_ms.append((t1 - t0) * 1e3)
        gm_ms.append((t2 - t1) * 1e3)
    rel = res[-1][1]
    out = {
        "metric": "Vanka cells·sweeps/s + GMRES time to 1e-8 rel. residual, FP32-patch vs FP64",
        "value": value, "unit": "cell-sweeps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32+f64", "bf16": "bf16+f32+f64", "f64": "f64"}[args.prec],
        "data": "synthetic (64 seeded Newton linearisations of channel flows; no dataset)",
        "config": {"workload": "batch64_seed0", "systems": len(B.systems), "unknowns": int(fin.n),
                   "finest_cells": int(B.n_cells_finest), "nnz_finest": int(fin.J.nnz),
                   "patch_sizes": sorted({g["n_K"] for g in fin.groups}), "packed_levels": len(B.levels),
                   "patch_precision": args.prec, "gmres_restart": restart, "nu_pre": nu[0], "nu_post": nu[1],
                   "omega": 0.7, "graphs": not args.no_graphs, "parallelism": "single GPU"},
        "performed_cell_sweeps_per_s": performed / dt,
        "gmres_iterations_per_system": [int(v) for v in its],
        "gmres_true_rel_residual_max": float(np.max(rel)),
        "setup_ms": float(np.median(setup_ms)), "gmres_ms_to_1e-8": float(np.median(gm_ms)),
        "eager_ms_per_step": dt_e / len(res_e) * 1e3, "graph_recordings_and_replays": list(graph_stats),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "patch_gemv (finest packed level, one launch per patch width)",
                     "bytes_per_sweep": bytes_sweep, "launches": n_apply,
                     "avg_sweep_ms": ms_apply / max(n_sweeps, 1)},
        "systems": [{"nx": s["shape"][0], "ny": s["shape"][1], "k": s["k"], "nu": s["nu"]} for s in B.systems],
    }
    S.close()
    if not args.no_cpu_baseline:
        # the FP64 oracle, one full step (setup + GMRES to 1e-8) of the first systems in turn
        t0 = time.perf_counter()
        cs = 0
        done = 0
        for si in range(len(B.systems)):
            H = oracle.OracleHierarchy(B.hierarchies[si])
            _, its_o, *_ = oracle.gmres(B.hierarchies[si][-1].J, B.rhs[si],
                                        lambda v, h=H: oracle.vcycle(h, v, *nu), restart=restart, rtol=1e-8)
            cs += its_o * sum(L.mesh.n_cells for L in B.hierarchies[si][1:]) * sum(nu)
            done += 1
            if time.perf_counter() - t0 > 15.0:
                break
        dt_c = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": cs / dt_c, "unit": "cell-sweeps/s", "cores": _threads(), "kind": "oracle",
                               "sample": f"one full step of systems 0..{done - 1} of the batch, {dt_c:.1f} s"}
    print(json.dumps(out), flush=True)


def run_learned(args, torch, vk, dev):
    """Learned initial guess on 200 consecutive dG(1) slabs of the 88 x 16 channel with a periodic
    inflow: slabs 1-100 are marched from the extrapolation guess, the BF16 network is trained on
    them (library kernels), and slabs 101-200 are marched three times to the same Newton tolerance
    (||F|| < 1e-8): from the extrapolation, from the raw learned guess, and from the judged guess
    (whichever of the two has the smaller slab residual).  Two inflows: the mild one of the
    workload (peak 0.3, period 0.5, one Newton step per slab) and a fast one (peak 1.0, period 0.1:
    ten slabs per period, two Newton steps per slab), where a better start can save a Newton step."""
    from synth.march import ChannelMarch
    from synth.learned import init_mlp_params, minibatch_orders, WIDTH, N_HIDDEN
    from paper_2210_02690_amd.guess import NewtonMarch, ExtrapolationGuess, LearnedGuess, JudgedGuess, march
    regimes = {"mild": (0.3, 0.5, 0.5), "fast": (1.0, 0.5, 0.1)}
    out = {
        "metric": "Newton and GMRES iterations and time over slabs 101-200 to ||F|| < 1e-8, judged learned guess "
                  "vs extrapolation",
        "unit": "s", "n_gpus": 1, "steps": 100, "warmup": 100, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 network + " + {"f32": "f32+f64", "bf16": "bf16+f32+f64",
                                                           "f64": "f64"}[args.prec] + " solver",
        "data": "synthetic (time-periodic channel inflow; no dataset)",
        "config": {"workload": "learned_guess_88x16", "mesh": [88, 16], "k": 1, "levels": 4, "slabs": 200,
                   "train_slabs": "1-100", "eval_slabs": "101-200", "epochs": args.epochs, "batch": 512,
                   "patch_precision": args.prec, "newton_tol": 1e-8, "gmres_rtol": 1e-8, "gmres_atol": 1e-10,
                   "inflows": {k: {"U0": v[0], "rel": v[1], "period": v[2]} for k, v in regimes.items()}},
    }
    for regime, inflow in regimes.items():
        t0 = time.perf_counter()
        pr = ChannelMarch(shape=(88, 16), levels=4, k=1, inflow=inflow)
        nm = NewtonMarch(pr, device=dev, prec=args.prec)
        fb = ExtrapolationGuess(pr, dev)
        slabs = [pr.initial_slab()]
        st_train = march(nm, 1, 100, slabs, fb)
        t_train_march = time.perf_counter() - t0
        log(f"[bench] {regime}: marched slabs 1-100 in {t_train_march:.1f} s")
        m = pr.fine.mesh
        lg = LearnedGuess(pr, WIDTH, N_HIDDEN, dev)
        n_samples = (len(slabs) - 2) * m.n_cells
        losses = lg.fit(slabs, init_mlp_params(2 * m.n_K, WIDTH, N_HIDDEN, m.n_K, seed=0),
                        minibatch_orders(n_samples, args.epochs, seed=0), batch=512, lr=1e-3)
        log(f"[bench] {regime}: trained {args.epochs} epochs on {n_samples} samples in {lg.train_seconds:.1f} s, "
            f"loss {losses[0]:.3e} -> {losses[-1]:.3e}")
        res = {}
        judged = JudgedGuess(lg, fb, pr)
        for name, guess in (("extrapolation", fb), ("learned", lg), ("judged", judged)):
            run = list(slabs)
            t1 = time.perf_counter()
            st = march(nm, 101, 200, run, guess)
            dt = time.perf_counter() - t1
            res[name] = {"seconds": dt, "newton_iterations": int(sum(s["newton"] for s in st)),
                         "gmres_iterations": int(sum(s["gmres"] for s in st)),
                         "mean_initial_residual": float(np.mean([s["F0"] for s in st])),
                         "median_initial_residual": float(np.median([s["F0"] for s in st])),
                         "all_converged": all(s["converged"] for s in st),
                         "seconds_assembly": float(sum(s["t_assembly"] for s in st)),
                         "seconds_solve": float(sum(s["t_solve"] for s in st)),
                         "seconds_residual": float(sum(s["t_residual"] for s in st)),
                         "seconds_guess": float(sum(s["t_guess"] for s in st)),
                         "final": run[-1]}
            log(f"[bench] {regime} {name}: newton {res[name]['newton_iterations']}, gmres "
                f"{res[name]['gmres_iterations']}, F0 mean {res[name]['mean_initial_residual']:.3e}, {dt:.1f} s")
        res["judged"]["choices"] = dict(judged.choices)
        ref = res["extrapolation"]["final"]
        for name in ("learned", "judged"):
            res[name]["rel_diff_slab200_vs_extrapolation"] = float(np.linalg.norm(res[name]["final"] - ref)
                                                                   / np.linalg.norm(ref))
        for name in res:
            res[name].pop("final")
        nm.close()
        out[regime] = dict(res, train={"march_seconds": t_train_march,
                                       "newton_iterations": int(sum(s["newton"] for s in st_train)),
                                       "gmres_iterations": int(sum(s["gmres"] for s in st_train)),
                                       "seconds": lg.train_seconds, "samples": n_samples,
                                       "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1]})
    out["value"] = out["fast"]["judged"]["seconds"]
    out["ms_per_step"] = out["value"] / 100 * 1e3
    print(json.dumps(out), flush=True)


def run_pmc_probe(args, torch, vk, dev):
    """Short fixed workload for hardware-counter runs (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE):
    three copies of a 512 MiB FP64 buffer (the calibration kernel: 512 MiB read and written per
    launch), then 20 finest-level additive sweeps of the workload with the same setup as the timed
    benchmark (each: SpMV, patch GEMV, DoF gather over the finest level)."""
    from synth import build_problem
    P = build_problem(args.config)
    S = vk.Solver([vk.upload_level(L, dev) for L in P.levels])
    S.vk_set_workspace(args.prec, 30, device=dev)
    S.vanka_setup(0.7, "additive")
    S.vk_autotune(10)
    n = (512 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    l = len(P.levels) - 1
    b = torch.from_numpy(P.b).to(dev)
    d = torch.zeros_like(b)
    S.vanka_smooth(l, b, d, 20, d_is_zero=False)
    torch.cuda.synchronize()
    print(json.dumps({"probe": args.config, "copy_bytes_per_launch": 2 * n * 8, "copy_launches": 3,
                      "sweeps": 20, "patch_gemv_bytes_per_launch": patch_gemv_bytes(P.finest, args.prec),
                      "spmv_bytes_per_launch": spmv_bytes(P.finest),
                      "spmv_stored_bytes_per_launch": S.vk_spmv_bytes(l),
                      "dof_gather_bytes_per_launch": gather_bytes(P.finest, args.prec),
                      "sweep_bytes": sweep_bytes(P.finest, args.prec),
                      "finest_cells": P.finest.mesh.n_cells}), flush=True)
    S.close()


def pmc_traffic(prec, config):
    """Measured HBM bytes of one finest-level sweep and of each of its kernels, from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration); None if the
    summary is missing, is for another workload, or the kernels' sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_sweep_{config}.json")
    csrc = os.path.join(ROOT, "paper_2210_02690_amd", "csrc")
    try:
        with open(path) as f:
            rec = json.load(f)
        digest = {}
        for name in ("sparse", "patch"):
            with open(os.path.join(csrc, f"{name}.hip"), "rb") as f:
                digest[name] = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("sparse_hip_sha256") != digest["sparse"] or rec.get("patch_hip_sha256") != digest["patch"]:
        return None
    return rec.get(prec)


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    except Exception:
        return 1


def run_robustness(args, torch, vk, dev):
    """Robustness in the time degree: one Newton linearisation per dG(k), k = 0..4 on the 88 x 16
    channel (Q2/P1disc, n_K = 21 (k + 1), and (Q4)^2/P3disc, the element of the paper's 2D study,
    n_K = 60 (k + 1)) and k = 0..2 on a 48 x 8 x 8 box (Q2/P1disc, n_K = 85 (k + 1)), each solved
    by GMRES(30) to 1e-8 with the two-plus-two-sweep V-cycle, FP64 and FP32 patch inverses.  The
    iteration counts are what the time degree should not change."""
    from synth import build_problem
    cases = [("channel2d_88x16", "channel2d_88x16_k1", dict(k=k)) for k in range(5)]
    cases += [("channel2d_88x16_q4", "channel2d_88x16_k1", dict(k=k, r=4)) for k in range(5)]
    cases += [("box3d_48x8x8", "box3d_100x16x16_k1", dict(shape=(48, 8, 8), levels=4, k=k)) for k in range(3)]
    restart, max_iter, nu = 30, 300, (2, 2)
    rows = []
    for name, cfg, over in cases:
        t0 = time.perf_counter()
        P = build_problem(cfg, **over)
        levels = [vk.upload_level(L, dev) for L in P.levels]
        b = torch.from_numpy(P.b).to(dev)
        x = torch.zeros_like(b)
        row = {"mesh": name, "r": int(P.finest.mesh.r), "k": over["k"], "n_K": int(P.finest.mesh.n_K),
               "unknowns": int(P.finest.n),
               "levels": len(P.levels), "coarse_unknowns": int(P.levels[0].n)}
        for prec in ("f64", "f32"):
            S = vk.Solver(levels)
            S.vk_set_workspace(prec, restart, device=dev)
            run_step(S, b, x, nu, restart, max_iter)  # warmup
            setup_ms, gmres_ms, its, rel = phase_times(torch, S, b, x, nu, restart, max_iter)
            xg = x.cpu().numpy()
            true_rel = float(np.linalg.norm(P.b - P.finest.J @ xg) / np.linalg.norm(P.b))
            row[prec] = {"gmres_iterations": int(its), "true_rel_residual": true_rel, "setup_ms": setup_ms,
                         "gmres_ms_to_1e-8": gmres_ms}
            S.close()
        rows.append(row)
        log(f"[bench] {name} k={over['k']} n_K={row['n_K']} n={row['unknowns']}: its f64 "
            f"{row['f64']['gmres_iterations']} f32 {row['f32']['gmres_iterations']} "
            f"({time.perf_counter() - t0:.1f} s)")
        del levels, b, x
        torch.cuda.empty_cache()
    out = {"metric": "GMRES(30) iterations to 1e-8 rel. residual per dG(k) linearisation, Vanka V-cycle "
                     "preconditioner (2+2 sweeps, omega 0.7)",
           "unit": "iterations", "n_gpus": 1, "higher_is_better": False, "data": "synthetic (seeded Newton "
           "linearisations of channel flows; no dataset)",
           "config": {"workload": "robustness_k", "restart": restart, "nu_pre": nu[0], "nu_post": nu[1]},
           "study": rows}
    print(json.dumps(out), flush=True)


def run_newton_march(args, torch, vk, dev):
    """Damped-Newton time marching with absolute tolerances (||F|| < 1e-8 per slab, GMRES to an
    absolute residual of 1e-9), dG(k) for k = 0..4 on the 88 x 16 channel with the periodic
    inflow, 20 slabs each from the extrapolated guess: Newton steps per slab and GMRES iterations
    per Newton step, the statistics of the paper's robustness tables."""
    from synth.march import ChannelMarch
    from paper_2210_02690_amd.guess import NewtonMarch, ExtrapolationGuess, march
    n_slabs = 20
    rows = []
    for k in range(5):
        t0 = time.perf_counter()
        pr = ChannelMarch(shape=(88, 16), levels=4, k=k)
        nm = NewtonMarch(pr, device=dev, prec=args.prec, tol=1e-8, rtol=0.0, atol=1e-9)
        slabs = [pr.initial_slab()]
        st = march(nm, 1, n_slabs, slabs, ExtrapolationGuess(pr, dev))
        nm.close()
        newton = sum(s["newton"] for s in st)
        gm = sum(s["gmres"] for s in st)
        row = {"k": k, "n_K": int(pr.fine.mesh.n_K), "unknowns": int(pr.n), "slabs": n_slabs,
               "newton_per_slab": newton / n_slabs, "gmres_per_newton": gm / max(newton, 1),
               "max_newton_per_slab": max(s["newton"] for s in st),
               "max_gmres_per_slab": max(s["gmres"] for s in st),
               "all_converged": all(s["converged"] for s in st),
               "final_residual_max": max(s["hist"][-1] for s in st),
               "seconds_solve": sum(s["t_solve"] for s in st), "seconds_total": time.perf_counter() - t0}
        rows.append(row)
        log(f"[bench] dG({k}) n_K={row['n_K']}: {row['newton_per_slab']:.2f} Newton/slab, "
            f"{row['gmres_per_newton']:.2f} GMRES/Newton, converged {row['all_converged']} "
            f"({row['seconds_total']:.1f} s)")
    out = {"metric": "Newton steps per slab and GMRES(30) iterations per Newton step, damped Newton with "
                     "absolute tolerances (||F|| < 1e-8, GMRES 1e-9)",
           "unit": "iterations", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic (88 x 16 channel with a periodic inflow, marched from Poiseuille flow)",
           "config": {"workload": "newton_march_k", "patch_precision": args.prec, "nu_pre": 2, "nu_post": 2,
                      "omega": 0.7, "tau": 0.01},
           "study": rows}
    print(json.dumps(out), flush=True)


def sweep_bytes(L, prec):
    """Algorithmic bytes of one additive sweep of level L that forms its defect (Eq. 3.5 with
    r = b - J d): N_c n_K^2 s_inv (the stored inverses) + nnz (8 + 4) (the CSR values and columns of
    J) + 4 (n + 1) (row pointers) + 3 * 8 n (b and d read, d written) + 4 N_c n_K (the cell -> DoF
    map).  The gathered defect entries and the per-DoF sums are taken as cache-resident."""
    nK, Nc, n = L.mesh.n_K, L.mesh.n_cells, L.n
    return Nc * nK * nK * PREC_BYTES[prec] + L.J.nnz * 12 + 4 * (n + 1) + 24 * n + 4 * Nc * nK


def spmv_bytes(L):
    """Algorithmic bytes of one defect r = b - J d on level L: values and columns, the int64 row
    pointers, d and b read once, r written."""
    return L.J.nnz * 12 + 8 * (L.n + 1) + 24 * L.n


def gather_bytes(L, prec):
    """Algorithmic bytes of one DoF gather d += omega z / p on level L: each cell product y_K entry
    read once (FP64 or FP32), the fixed-width cell lists (8 int32 per DoF in 3D, 4 in 2D), 1/p read,
    d read and written."""
    w = 8 if L.mesh.d == 3 else 4
    sy = 8 if prec == "f64" else 4
    return L.mesh.n_cells * L.mesh.n_K * sy + L.n * (4 * w + 24)


def roofline_entry(bound, achieved, peak, unit, **extra):
    out = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak}
    out.update(extra)
    return out


FP64_PEAK_TFS = 78.6   # MI355X FP64 (vector and matrix), TFLOP/s


def measure(torch, vk, S, P, b, x, nu, restart, max_iter, steps, warmup, prec, label):
    """Warm-up, then `steps` timed steps (setup + GMRES to 1e-8) with the finest level's sweeps,
    SpMV, patch GEMV, DoF gather and patch inversion timed by HIP events inside the timed region;
    then the block inversion of the coarsest level from two more steps.  Returns the record."""
    L = len(P.levels) - 1
    fine = P.finest
    cs_per_vc = cells_sweeps_per_vcycle(P, *nu)
    for w in range(warmup):
        its, rel = run_step(S, b, x, nu, restart, max_iter)
        log(f"[bench] {label} warmup {w}: {its} its, rel {rel:.2e}")
    kinds = ["sweep", "spmv", "patch_gemv", "dof_gather", "patch_setup"]
    # A 2D step is a few ms of short launches: events on every bracketed launch would cost about
    # 1 ms per step there, so one bracketed launch in seven is timed (7 is prime to the four sweeps
    # per level and V-cycle, so every sweep position is sampled).  3D launches last 0.03-1 ms: all.
    S.vk_timing_kinds(kinds, every=7 if fine.mesh.d == 2 else 1)
    S.vk_timing_enable(True, L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_its = 0
    for _ in range(steps):
        its, rel = run_step(S, b, x, nu, restart, max_iter)
        total_its += its
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    live = {k: S.vk_timing_read(k, L) for k in kinds}
    S.vk_timing_kinds(["block_invert"])
    S.vk_timing_enable(True, 0)
    for _ in range(2):
        run_step(S, b, x, nu, restart, max_iter)
    live["block_invert"] = S.vk_timing_read("block_invert", 0)
    S.vk_timing_enable(False)
    S.vk_timing_kinds(None)
    avg = {k: (ms / n if n else None) for k, (n, ms) in live.items()}
    log(f"[bench] {label}: timed {steps} steps in {dt:.3f} s, {total_its} GMRES its; finest sweep "
        f"{avg['sweep']} ms, spmv {avg['spmv']} ms, gemv {avg['patch_gemv']} ms, setup {avg['patch_setup']} ms")
    bs = sweep_bytes(fine, prec)
    sweep_gbs = bs / (avg["sweep"] * 1e-3) / 1e9
    # bytes the finest J actually occupies in the storage in use (grouped CSR shares column lists,
    # so it moves less than the CSR figure the roofline is defined on)
    lf = len(P.levels) - 1
    stored = S.vk_spmv_bytes(lf)
    lpr_g = S.vk_spmv_format(lf)
    kern = {
        "spmv": roofline_entry("hbm", spmv_bytes(fine) / (avg["spmv"] * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s",
                               bytes_per_launch=spmv_bytes(fine), avg_launch_ms=avg["spmv"],
                               launches=live["spmv"][0],
                               storage=(f"grouped CSR, {lpr_g} lanes per group" if lpr_g else "CSR"),
                               stored_bytes_per_launch=stored,
                               stored_gbs=stored / (avg["spmv"] * 1e-3) / 1e9),
        "patch_gemv": roofline_entry("hbm", patch_gemv_bytes(fine, prec) / (avg["patch_gemv"] * 1e-3) / 1e9,
                                     HBM_PEAK_GBS, "GB/s", bytes_per_launch=patch_gemv_bytes(fine, prec),
                                     avg_launch_ms=avg["patch_gemv"], launches=live["patch_gemv"][0]),
        "dof_gather": roofline_entry("hbm", gather_bytes(fine, prec) / (avg["dof_gather"] * 1e-3) / 1e9,
                                     HBM_PEAK_GBS, "GB/s", bytes_per_launch=gather_bytes(fine, prec),
                                     avg_launch_ms=avg["dof_gather"], launches=live["dof_gather"][0]),
    }
    flops_setup = 2.0 * fine.mesh.n_K ** 3 * fine.mesh.n_cells
    if avg["patch_setup"]:
        kern["patch_setup"] = roofline_entry("alu", flops_setup / (avg["patch_setup"] * 1e-3) / 1e12, FP64_PEAK_TFS,
                                             "TFLOP/s", flops_per_launch=flops_setup,
                                             avg_launch_ms=avg["patch_setup"], launches=live["patch_setup"][0],
                                             note="finest-level patch gather + FP64 Gauss-Jordan inversions, "
                                                  "2 n_K^3 flop per cell")
    n0 = P.levels[0].n
    if avg["block_invert"]:
        nb, fl = S.vk_coarse_plan(0)
        what = (f"block-tridiagonal factorisation of the coarsest level's {n0} unknowns in {nb} level-set "
                f"blocks (dense Gauss-Jordan inverses of the Schur-complement blocks and the coupling "
                f"products)") if nb > 0 else f"FP64 Gauss-Jordan inverse of the coarsest level's {n0} unknowns"
        kern["block_invert"] = roofline_entry("mfma" if nb == 0 else "alu", fl / (avg["block_invert"] * 1e-3) / 1e12,
                                              FP64_PEAK_TFS, "TFLOP/s", flops_per_launch=fl,
                                              avg_ms=avg["block_invert"], blocks=nb,
                                              note=what + ": a chain of launches, bracketed as one")
    setup_ms, gmres_ms, its_h, rel_h = phase_times(torch, S, b, x, nu, restart, max_iter)
    # HBM bytes per launch from the committed counter summary (None when it does not apply)
    tr = pmc_traffic(prec, P.name)
    traffic = tr["sweep_traffic_bytes"] if tr else None
    if tr:
        for k, rec in tr["kernels"].items():
            for name in kern:
                if k.startswith(name):
                    kern[name]["traffic"] = rec["traffic_bytes"]
    return {
        "value": total_its * cs_per_vc / dt, "ms_per_step": dt / steps * 1e3, "steps": steps,
        "gmres_iterations": its_h, "gmres_true_rel_residual": rel_h, "gmres_ms_to_1e-8": gmres_ms,
        "setup_ms": setup_ms,
        "roofline": roofline_entry("hbm", sweep_gbs, HBM_PEAK_GBS, "GB/s",
                                   kernel="whole finest-level additive sweep with its defect (SpMV + patch GEMV "
                                          "+ DoF gather), bracketed by events as one unit",
                                   traffic=traffic, bytes_per_sweep=bs,
                                   stored_bytes_per_sweep=bs - spmv_bytes(fine) + stored,
                                   avg_sweep_ms=avg["sweep"],
                                   sweeps=live["sweep"][0], kernels=kern),
        "finest_cell_sweeps_per_s": fine.mesh.n_cells / (avg["sweep"] * 1e-3),
    }


def cpu_baseline_protocol(P, nu, restart, cs_per_vc, its_gpu):
    """The FP64 oracle timed phase by phase on a bounded sample of the same workload, median of 5
    after one warm-up, on one core and on all cores:
      setup_per_cell: patch gather + LAPACK inverse of 16 finest cells, per cell;
      spmv: r = b - J d with the whole finest J (the defect of one sweep);
      patch_apply_per_cell: the einsum of A_K r_K and its scatter for 1 024 cells (the 16 sampled
        inverses repeated: the cost depends on the shapes only), per cell;
      coarse_lu: LU factorisation of the dense coarsest matrix (all cores only).
    value = finest-level cell-sweeps/s of the oracle's additive sweep, spmv + N_c * patch_apply
    (all cores); step_estimate_s = setup (every level's cells + coarse LU) + GMRES iterations x
    V-cycle sweeps (the sweeps dominate the oracle's V-cycle), with the GPU's iteration count."""
    import platform
    import oracle
    from threadpoolctl import threadpool_limits
    fine = P.finest
    J = fine.J
    cd = fine.cell_dofs
    rng = np.random.default_rng(3)
    cells = np.sort(rng.choice(fine.mesh.n_cells, 16, replace=False))
    rep = np.resize(cells, 1024)
    d = rng.standard_normal(fine.n)
    r = P.b - J @ d
    A16 = None

    def med(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    def setup16():
        nonlocal A16
        A16 = oracle.invert_patches(oracle.patch_matrices(J, cd[cells]))

    def apply1024():
        A = A16[np.arange(1024) % 16]
        y = np.einsum("kij,kj->ki", A, r[cd[rep]])
        z = np.zeros(fine.n)
        np.add.at(z, cd[rep].ravel(), y.ravel())

    J0 = P.levels[0].J.toarray()
    out = {}
    for cores in ("1", "all"):
        lim = 1 if cores == "1" else None
        with threadpool_limits(limits=lim):
            ph = {"setup_per_cell_ms": med(setup16) / 16 * 1e3,
                  "spmv_ms": med(lambda: P.b - J @ d) * 1e3,
                  "patch_apply_per_cell_ms": med(apply1024) / 1024 * 1e3}
            if cores == "all":
                import scipy.linalg as sla
                ph["coarse_lu_ms"] = med(lambda: sla.lu_factor(J0), reps=3) * 1e3
        out[cores] = ph
    a = out["all"]
    sweep_s = (a["spmv_ms"] + a["patch_apply_per_cell_ms"] * fine.mesh.n_cells) * 1e-3
    cells_all = sum(L.mesh.n_cells for L in P.levels[1:])
    setup_s = a["setup_per_cell_ms"] * cells_all * 1e-3 + a["coarse_lu_ms"] * 1e-3
    vcycle_s = sum((sum(nu)) * (a["spmv_ms"] * L.J.nnz / J.nnz + a["patch_apply_per_cell_ms"] * L.mesh.n_cells)
                   * 1e-3 for L in P.levels[1:])
    step_s = setup_s + its_gpu * vcycle_s
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = platform.processor()
    try:
        from threadpoolctl import threadpool_info
        threads = int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    except Exception:
        threads = 1
    return {"value": fine.mesh.n_cells / sweep_s, "unit": "cell-sweeps/s", "cores": threads, "kind": "oracle",
            "sample": "finest-level additive sweep of the same workload from timed parts: the SpMV with the "
                      "whole J, and the patch apply of 1 024 cells scaled to all cells (median of 5 after a "
                      "warm-up, all cores)",
            "phases_1_core": out["1"], "phases_all_cores": out["all"], "cpu_model": model,
            "nproc": os.cpu_count(), "step_estimate_s": step_s,
            "step_estimate_cell_sweeps_per_s": its_gpu * cs_per_vc / step_s,
            "step_estimate": "setup of every level's patches + coarse LU + GMRES iterations (the GPU's count) "
                             "x V-cycle sweeps, from the phase timings"}


def run_extra_channel(torch, vk, dev, nu, restart, max_iter, steps):
    """The 176 x 32 dG(2) channel (5 levels, n_K = 63): FP32, FP64 and BF16 inverses."""
    from synth import build_problem
    P = build_problem("channel2d_176x32_k2")
    levels = [vk.upload_level(L, dev) for L in P.levels]
    b = torch.from_numpy(P.b).to(dev)
    x = torch.zeros_like(b)
    cs_per_vc = cells_sweeps_per_vcycle(P, *nu)
    out = {"workload": "channel2d_176x32_k2", "unknowns": int(P.finest.n), "finest_cells": int(P.finest.mesh.n_cells),
           "patch_size": int(P.finest.mesh.n_K)}
    for prec in ("f32", "f64", "bf16"):
        S = vk.Solver(levels)
        S.vk_set_workspace(prec, restart, device=dev)
        S.vanka_setup(0.7, "additive")
        S.vk_autotune(10)
        for _ in range(3):
            run_step(S, b, x, nu, restart, max_iter)
        dt, res = timed_steps(torch, lambda: run_step(S, b, x, nu, restart, max_iter), steps)
        s_ms, g_ms, its, rel = phase_times(torch, S, b, x, nu, restart, max_iter)
        out[prec] = {"value": sum(r[0] for r in res) * cs_per_vc / dt, "ms_per_step": dt / steps * 1e3,
                     "setup_ms": s_ms, "gmres_ms_to_1e-8": g_ms, "gmres_iterations": its,
                     "gmres_true_rel_residual": rel,
                     "finest_cell_sweeps_per_s": sweep_rate(torch, S, P, P.b)}
        S.close()
        log(f"[bench] channel 176x32 {prec}: {out[prec]['ms_per_step']:.2f} ms/step, {its} its")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="box3d_100x16x16_k1")
    ap.add_argument("--prec", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 leg and the 2D channel figures")
    ap.add_argument("--compare-precs", default="f64", help="precisions of the comparison legs")
    ap.add_argument("--no-graphs", action="store_true", help="batch: launch Arnoldi steps eagerly")
    ap.add_argument("--epochs", type=int, default=40, help="learned guess: training epochs")
    ap.add_argument("--pmc-probe", action="store_true", help="short fixed workload for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2210_02690_amd as vk
    from synth import build_problem

    dev = torch.device("cuda:0")
    # The workload runs on a stream of its own (default priority), as a serving loop would: on the
    # legacy default stream every launch would also wait for the library's CU-masked setup stream
    # (a blocking stream), so the coarser levels' patch inversions could not overlap the solve.
    torch.cuda.set_stream(torch.cuda.Stream(dev))
    if args.config == "batch64_seed0":
        return run_batch(args, torch, vk, dev)
    if args.config == "learned_guess_88x16":
        return run_learned(args, torch, vk, dev)
    if args.config == "robustness_k":
        return run_robustness(args, torch, vk, dev)
    if args.config == "newton_march_k":
        return run_newton_march(args, torch, vk, dev)
    if args.pmc_probe:
        return run_pmc_probe(args, torch, vk, dev)
    restart, max_iter, nu = 30, 300, (2, 2)
    t0 = time.perf_counter()
    P = build_problem(args.config)
    log(f"[bench] built {args.config}: n = {P.finest.n}, levels = {len(P.levels)}, "
        f"{time.perf_counter() - t0:.1f} s")
    levels = [vk.upload_level(L, dev) for L in P.levels]
    b = torch.from_numpy(P.b).to(dev)
    x = torch.zeros_like(b)
    fine = P.finest

    def make(prec):
        S = vk.Solver(levels)
        S.vk_set_workspace(prec, restart, device=dev)
        S.vanka_setup(0.7, "additive")
        S.vk_autotune(10)
        return S

    S = make(args.prec)
    head = measure(torch, vk, S, P, b, x, nu, restart, max_iter, args.steps, args.warmup, args.prec, args.prec)
    x_head = x.cpu().numpy()
    gmres_x_true = float(np.linalg.norm(P.b - fine.J @ x_head) / np.linalg.norm(P.b))
    # the same steps with every Arnoldi step replayed from a recorded hipGraph
    S.vk_set_graphs(True)
    run_step(S, b, x, nu, restart, max_iter)  # records the step graphs
    reps = max(5, args.steps // 2)
    dt_g, res = timed_steps(torch, lambda: run_step(S, b, x, nu, restart, max_iter), reps)
    s_ms, g_ms, its_g, rel_g = phase_times(torch, S, b, x, nu, restart, max_iter)
    graphs = {"value": sum(r[0] for r in res) * cells_sweeps_per_vcycle(P, *nu) / dt_g,
              "ms_per_step": dt_g / reps * 1e3, "gmres_ms_to_1e-8": g_ms, "setup_ms": s_ms,
              "gmres_iterations": its_g,
              "rel_diff_solution_vs_eager": float(np.linalg.norm(x.cpu().numpy() - x_head) / np.linalg.norm(x_head)),
              "graph_recordings": S.vk_graph_stats()[0]}
    log(f"[bench] graphs: {dt_g / reps * 1e3:.2f} ms/step, gmres {g_ms:.2f} ms")
    S.vk_set_graphs(False)
    S.close()
    cg, rg = stream_rates_gbs(torch, dev)
    rf = head.pop("roofline")
    rf["copy_GBps"] = cg
    rf["read_GBps"] = rg
    rf["frac_of_read"] = rf["achieved"] / rg
    out = {
        "metric": "Vanka cells·sweeps/s + GMRES time to 1e-8 rel. residual, FP32-patch vs FP64",
        "value": head["value"], "unit": "cell-sweeps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32+f64", "bf16": "bf16+f32+f64", "f64": "f64"}[args.prec],
        "data": "synthetic (seeded Newton linearisation of a channel/box flow; no dataset)",
        "config": {"workload": args.config, "unknowns": int(fine.n), "levels": len(P.levels),
                   "finest_cells": int(fine.mesh.n_cells), "patch_size": int(fine.mesh.n_K),
                   "nnz_finest": int(fine.J.nnz), "patch_precision": args.prec, "gmres_restart": restart,
                   "nu_pre": nu[0], "nu_post": nu[1], "omega": 0.7, "parallelism": "single GPU"},
        "gmres_iterations": head["gmres_iterations"], "gmres_true_rel_residual": head["gmres_true_rel_residual"],
        "gmres_true_rel_residual_host": gmres_x_true,
        "gmres_ms_to_1e-8": head["gmres_ms_to_1e-8"], "setup_ms": head["setup_ms"],
        "finest_cell_sweeps_per_s": head["finest_cell_sweeps_per_s"],
        "roofline": rf, "graphs": graphs,
    }
    if not args.no_compare:
        for prec in [q for q in args.compare_precs.split(",") if q and q != args.prec]:
            S2 = make(prec)
            rec = measure(torch, vk, S2, P, b, x, nu, restart, max_iter, max(3, args.steps // 2), 1, prec, prec)
            xs = x.cpu().numpy()
            rec["rel_diff_solution_vs_headline"] = float(np.linalg.norm(xs - x_head) / np.linalg.norm(xs))
            rec["gmres_ms_ratio_vs_headline"] = rec["gmres_ms_to_1e-8"] / head["gmres_ms_to_1e-8"]
            out[prec] = rec
            S2.close()
            log(f"[bench] {prec}: {rec['gmres_iterations']} its, gmres {rec['gmres_ms_to_1e-8']:.2f} ms, "
                f"sweep frac {rec['roofline']['frac']:.3f}")
        if args.config != "channel2d_176x32_k2":
            del levels
            torch.cuda.empty_cache()
            out["channel2d_176x32_k2"] = run_extra_channel(torch, vk, dev, nu, restart, max_iter,
                                                           max(5, args.steps // 2))
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline_protocol(P, nu, restart, cells_sweeps_per_vcycle(P, *nu),
                                                    head["gmres_iterations"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
