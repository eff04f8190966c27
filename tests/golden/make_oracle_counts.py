"""Write tests/golden/oracle_counts.json: GMRES iteration counts of the FP64 CPU oracle at the
workloads' full sizes, which the GPU parity tests compare against (counts within +-1).

Imports only oracle/ and synth/ (the seeded input generators); nothing here touches the HIP
library.  Each entry is one oracle GMRES(30) solve, right-preconditioned by the V-cycle with
additive coloured Vanka (omega = 0.7), from x0 = 0 to a relative residual of 1e-8 (Sec. 3; the
stopping rule of the oracle's gmres), with the patch inverses stored as given by `prec`:
  f64   the LAPACK inverses themselves;
  f32   each inverse rounded to FP32 (round to nearest even), applied in FP64 arithmetic;
  bf16  each inverse rounded to BF16 (RNE), applied in FP64 arithmetic.
The rounded cases are the project's mixed-precision extension: the oracle applies exactly the
stored values the GPU applies, so the counts compare like with like (the GPU accumulates in FP32,
which the +-1 tolerance absorbs).

Usage (from the repository root):
  python tests/golden/make_oracle_counts.py [part ...]
parts: cfg1, cfg1_nu44, cfg0_nu44, box3d (V-cycle sample, both precisions), box3d_f64, box3d_f32, batch64, all.  Each part merges
its entries into the JSON file, so parts may run in separate processes.
"""
import fcntl
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import build_problem  # noqa: E402

OUT = os.path.join(HERE, "oracle_counts.json")
STORE = {"f64": None, "f32": oracle.round_f32, "bf16": oracle.round_bf16}


def _solve(levels, b, prec, nu=(2, 2)):
    H = oracle.OracleHierarchy(levels, patch_store=STORE[prec])
    t0 = time.perf_counter()
    x, its, hist, conv, true_rel = oracle.gmres(levels[-1].J, b, lambda v: oracle.vcycle(H, v, *nu),
                                                restart=30, max_iter=300, rtol=1e-8)
    dt = time.perf_counter() - t0
    return dict(iters=int(its), converged=bool(conv), true_rel=float(true_rel),
                history=[float(h) for h in hist], seconds=round(dt, 1))


def _merge(entries):
    # parts may run in parallel processes: read-modify-write under an exclusive lock
    with open(OUT + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        _merge_locked(entries)


def _merge_locked(entries):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_command"] = "python tests/golden/make_oracle_counts.py [part ...]"
    data["_what"] = ("oracle GMRES(30) + V-cycle(nu_pre, nu_post) + additive coloured Vanka, omega 0.7, "
                     "x0 = 0, rtol 1e-8; patch inverses stored as f64 / rounded to f32 / bf16")
    data.setdefault("entries", {}).update(entries)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


def part_problem(name, precs, nu=(2, 2)):
    P = build_problem(name)
    ent = {}
    for prec in precs:
        r = _solve(P.levels, P.b, prec, nu)
        key = f"{name}/{prec}/nu{nu[0]}{nu[1]}"
        print(f"{key}: {r['iters']} its, true rel {r['true_rel']:.3e}, {r['seconds']} s", flush=True)
        ent[key] = r
        _merge({key: r})
    return ent


def part_box3d():
    """The 3D box: V(b) at seeded sample indices (FP64 inverses), then GMRES with FP64 and with
    FP32-rounded inverses.  The hierarchies are built one after the other (each holds 5.9 GB of
    patch inverses)."""
    name = "box3d_100x16x16_k1"
    P = build_problem(name)
    H = oracle.OracleHierarchy(P.levels)
    t0 = time.perf_counter()
    v = oracle.vcycle(H, P.b, 2, 2)
    idx = np.sort(np.random.default_rng(7).choice(P.finest.n, 2000, replace=False))
    ent = {"indices": [int(i) for i in idx], "values": [float(x) for x in v[idx]],
           "max_abs": float(np.abs(v).max()), "norm2": float(np.linalg.norm(v)),
           "seconds": round(time.perf_counter() - t0, 1)}
    _merge({f"{name}/f64/vcycle22_sample": ent})
    print(f"{name} V-cycle sample written ({ent['seconds']} s)", flush=True)
    del H, v
    for prec in ("f64", "f32"):
        r = _solve(P.levels, P.b, prec)
        key = f"{name}/{prec}/nu22"
        print(f"{key}: {r['iters']} its, true rel {r['true_rel']:.3e}, {r['seconds']} s", flush=True)
        _merge({key: r})


def part_batch64(precs=("f32", "f64")):
    from synth.batch import build_batch
    B = build_batch(64, seed=0)
    for prec in precs:
        ent = {}
        for si, h in enumerate(B.hierarchies):
            r = _solve(h, B.rhs[si], prec)
            r.pop("history")
            ent[str(si)] = r
            print(f"batch64_seed0/{prec}/{si}: {r['iters']} its ({r['seconds']} s)", flush=True)
        _merge({f"batch64_seed0/{prec}/nu22": ent})


PARTS = {
    "cfg1": lambda: part_problem("channel2d_176x32_k2", ("f64", "f32", "bf16")),
    "cfg1_nu44": lambda: part_problem("channel2d_176x32_k2", ("f64", "f32"), nu=(4, 4)),
    "cfg0_nu44": lambda: part_problem("channel2d_44x8_k1", ("f64",), nu=(4, 4)),
    "box3d": part_box3d,
    "box3d_f64": lambda: part_problem("box3d_100x16x16_k1", ("f64",)),
    "box3d_f32": lambda: part_problem("box3d_100x16x16_k1", ("f32",)),
    "batch64": part_batch64,
}

if __name__ == "__main__":
    parts = sys.argv[1:] or ["all"]
    if parts == ["all"]:
        parts = ["cfg1", "cfg1_nu44", "cfg0_nu44", "box3d", "batch64"]
    for p in parts:
        PARTS[p]()
