"""The stored oracle results in tests/golden/oracle_counts.json are the oracle's own: the cheapest
entries are recomputed here from the oracle and the seeded generators and must agree exactly, and
every stored solve reached the tolerance its entry names (true relative residual <= 1e-8)."""
import json
import os

import numpy as np
import pytest

import oracle
from synth import build_problem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_counts.json")


def _entries():
    with open(GOLDEN) as f:
        return json.load(f)["entries"]


def test_cheap_entry_recomputes_exactly():
    ent = _entries()["channel2d_44x8_k1/f64/nu44"]
    P = build_problem("channel2d_44x8_k1")
    H = oracle.OracleHierarchy(P.levels)
    _, its, hist, conv, rel = oracle.gmres(P.finest.J, P.b, lambda v: oracle.vcycle(H, v, 4, 4),
                                          restart=30, max_iter=300, rtol=1e-8)
    assert conv and its == ent["iters"]
    assert np.allclose(hist, ent["history"], rtol=1e-12, atol=0.0)


def test_stored_solves_converged():
    for key, ent in _entries().items():
        if key.startswith("batch64"):
            for si, e in ent.items():
                assert e["converged"] and e["true_rel"] <= 1e-8, (key, si)
        elif "iters" in ent:
            assert ent["converged"] and ent["true_rel"] <= 1e-8, key
            h = np.asarray(ent["history"])
            assert len(h) == ent["iters"] + 1 and h[-1] <= 1e-8 * h[0] * (1 + 1e-12), key


def test_required_entries_present():
    ent = _entries()
    need = ["channel2d_176x32_k2/f64/nu22", "channel2d_176x32_k2/f32/nu22", "channel2d_176x32_k2/bf16/nu22",
            "channel2d_176x32_k2/f64/nu44", "channel2d_176x32_k2/f32/nu44", "box3d_100x16x16_k1/f64/nu22",
            "box3d_100x16x16_k1/f32/nu22", "box3d_100x16x16_k1/f64/vcycle22_sample", "batch64_seed0/f32/nu22"]
    missing = [k for k in need if k not in ent]
    assert not missing, missing
    assert len(ent["batch64_seed0/f32/nu22"]) == 64
