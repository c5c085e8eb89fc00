"""Full-length runs against stored oracle summaries.

tests/golden/long_runs.json is written by tests/golden/make_long_runs.py,
which runs only the CPU oracle (FP64) for the whole step count and keeps, at
each snapshot, the sums of phi and phi^2, block means over a coarse grid and
phi at seeded sample nodes.  Here the GPU path runs the same workload from the
same seeded phi0, in the launch configuration the benchmark uses (autotuned:
tile shape, block order, graph replays or direct launches), and the same
summaries are compared:

    FP64 storage   samples / block means relative L2 <= 1e-12, sums <= 1e-12
    FP32 offsets   <= 1e-5
    FP16 offsets   reported, with loose per-workload bounds (see TOL)

Workloads: the nonlinear anisotropic D2Q9 case with the Scheme-A source at
its full 1024 x 1024 size and 5000 steps, the same in Scheme B (Eq. 35
implicit in phi), and the same between walls with unequal non-flux rates
(the moment-space collision); the D3Q19 case with walls, at the full 2000
steps on 64^3 and 128^3 grids and for the first 200 steps on its full 256^3
grid (the whole 256^3 run would take the host oracle hours), and on 128^3
with a Scheme-A source and K(phi) for 1000 steps.  Beside the relative L2 of
the samples, the largest
sample difference relative to the largest |phi| of the samples is bounded by
the same tolerance.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_runs.json")
# FP16 bounds are loose sanity bounds on a reported figure: the 2-D workload
# is re-centred (it has a source) and ends near 5e-4; the D3Q19 field keeps
# O(1) structure on a zero background, so its stored values cannot be made
# small and 10-bit rounding accumulates to about 4e-3 over 2000 steps.  Between
# walls held at 0.3 and 0.7 the 2-D field keeps offsets of about 0.3 from any
# reference, and FP16 rounding accumulates to about 2e-2 over 5000 steps.
TOL = {"f64": 1e-12, "f32": 1e-5, ("nonlinear2d-1024", "f16"): 2e-3, ("d3q19-walls-64", "f16"): 1e-2,
       ("d3q19-walls-128", "f16"): 1e-2, ("nonlinear2d-1024-scheme-b", "f16"): 2e-3,
       ("nonlinear2d-1024-walls-rates", "f16"): 6e-2, ("d3q19-128-source", "f16"): 2e-2,
       ("d3q19-walls-256", "f16"): 1e-2}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def load():
    if not os.path.exists(GOLDEN):
        pytest.fail(f"{GOLDEN} missing: run tests/golden/make_long_runs.py")
    return json.load(open(GOLDEN))


def workload(name, precision):
    if name == "nonlinear2d-1024":
        spec, phi0, _ = W.nonlinear_2d(1024, precision=precision)
    elif name == "nonlinear2d-1024-scheme-b":
        spec, phi0, _ = W.nonlinear_2d(1024, precision=precision)
        spec["scheme"] = "B"
    elif name == "d3q19-walls-64":
        spec, phi0, _ = W.d3q19_walls((64, 64, 64), precision=precision)
    elif name == "d3q19-walls-128":
        spec, phi0, _ = W.d3q19_walls((128, 128, 128), precision=precision)
    elif name == "nonlinear2d-1024-walls-rates":
        spec, phi0, _ = W.nonlinear_2d_walls_rates(1024, precision=precision)
    elif name == "d3q19-128-source":
        spec, phi0, _ = W.d3q19_walls_source((128, 128, 128), precision=precision)
    elif name == "d3q19-walls-256":
        spec, phi0, _ = W.d3q19_walls((256, 256, 256), precision=precision)
    else:
        raise KeyError(name)
    return spec, phi0


def summaries(phi, edge, idx):
    f = phi.double()
    shp = []
    for n in f.shape:
        shp += [n // edge, edge]
    blocks = f.reshape(shp).mean(dim=tuple(range(1, 2 * f.dim(), 2))).reshape(-1)
    flat = f.reshape(-1)
    return (float(f.sum()), float((f * f).sum()), blocks.cpu().numpy(),
            flat[torch.as_tensor(idx, device=flat.device)].cpu().numpy())


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
@pytest.mark.parametrize("name", ["nonlinear2d-1024", "d3q19-walls-64", "d3q19-walls-128",
                                  "nonlinear2d-1024-scheme-b", "nonlinear2d-1024-walls-rates",
                                  "d3q19-128-source", "d3q19-walls-256"])
def test_full_length_against_oracle(name, precision):
    from paper_1603_09577_amd import lbm
    g = load().get(name)
    if g is None:
        pytest.fail(f"{name} missing from {GOLDEN}: run tests/golden/make_long_runs.py --cases {name}")
    spec, phi0 = workload(name, precision)
    assert list(phi0.shape) == g["shape"]
    sim = lbm.Lbm(spec).init(phi0)
    sim.tune(reps=5)          # the launch configuration the benchmark times
    tol = TOL.get((name, precision), TOL.get(precision))
    t = 0
    worst = 0.0
    for s in sorted(int(k) for k in g["snapshots"]):
        sim.step(s - t)
        t = s
        ref = g["snapshots"][str(s)]
        gs, gq, gb, gv = summaries(sim.phi(), g["block_edge"], g["idx"])
        e_vals = rel(gv, ref["vals"])
        e_pt = float(np.abs(np.asarray(gv) - np.asarray(ref["vals"])).max() / np.abs(np.asarray(ref["vals"])).max())
        e_blk = rel(gb, ref["blocks"])
        e_sum = abs(gs - ref["sum"]) / abs(ref["sum"])
        e_sq = abs(gq - ref["sumsq"]) / abs(ref["sumsq"])
        say(f"[gpu long run] {name} {precision} step {s}: samples {e_vals:.2e} (pointwise {e_pt:.2e}) "
            f"blocks {e_blk:.2e} sum {e_sum:.2e} sumsq {e_sq:.2e}")
        worst = max(worst, e_vals, e_pt, e_blk, e_sum, e_sq)
    assert worst <= tol, f"{name} {precision}: {worst:.3e} > {tol}"
