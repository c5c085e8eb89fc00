"""Time-dependent Dirichlet walls (anti-bounce-back, Sec. 3.6) on the GPU
against the oracle.

The oracle streams in push form: its step t applies the wall values phi_w(t).
The GPU stores post-collision values and streams them in the gather of the
next sweep, so phi_w(t) is set right after the sweep of step t (and the first
gather after initialisation sees the values the initialisation saw).
FP64 <= 1e-12 relative L2, FP32 <= 1e-5.
"""
import math
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def schedule(t, T):
    return 0.3 + 0.1 * math.sin(2 * math.pi * t / 40.0), 0.7 - 0.2 * t / T


def oracle_run(spec, phi0, T, wall_of):
    p = orc.params_from_spec(dict(spec, precision="f64"))
    axis = 1 if spec["lattice"] == 9 else 2
    f, pp = orc.init(p, phi0)
    for t in range(T):
        lo, hi = wall_of(t)
        p.phi_wall[axis][0], p.phi_wall[axis][1] = lo, hi
        orc.step(p, f, pp)
    return orc.phi(p, f)


def compare(name, spec, phi0, T, tol):
    from paper_1603_09577_amd import lbm
    say(f"[gpu walls] {name} shape={spec['shape']} prec={spec.get('precision', 'f64')} T={T}")
    sim = lbm.Lbm(spec).init(phi0)
    for t in range(T):
        sim.step(1)
        sim.set_phi_wall(*schedule(t, T))
    got = sim.phi().cpu().numpy()
    ref = oracle_run(spec, phi0, T, lambda t: schedule(t, T))
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    say(f"    rel L2 vs oracle {e:.2e}")
    assert e <= tol


def _spec2(nx, ny, precision="f64"):
    spec = W.spec_nonlinear_2d(nx, ny, precision=precision)
    spec["bc"] = ["periodic", "abb", "periodic"]
    spec["phi_wall"] = [[0, 0], [0.3, 0.7], [0, 0]]
    return spec


def test_time_dependent_walls_d2q9():
    compare("D2Q9 nonlinear", _spec2(25, 19), W.noise_field((19, 25), 61), 90, 1e-12)


def test_time_dependent_walls_d2q9_fp32():
    compare("D2Q9 nonlinear fp32", _spec2(25, 19, "f32"), W.noise_field((19, 25), 62), 90, 1e-5)


def test_time_dependent_walls_d3q19():
    n = (10, 9, 13)
    spec = W.spec_d3q19_aniso(n, phi_wall=0.3)
    compare("D3Q19", spec, W.gaussians_3d(n, 11), 50, 1e-12)


def test_wall_values_between_graph_replays():
    """Values changed between runs of 32 graph-replayed sweeps: the gathers of
    sweeps 32 b ... 32 b + 31 stream steps 32 b - 1 ... 32 b + 30, so the
    oracle's schedule changes one step before each block."""
    from paper_1603_09577_amd import lbm
    spec = _spec2(40, 33)
    phi0 = W.noise_field((33, 40), 63)
    vals = [(0.3, 0.7), (0.5, 0.6), (0.2, 0.9), (0.4, 0.4)]
    sim = lbm.Lbm(spec).init(phi0)
    for b, v in enumerate(vals):
        if b:
            sim.set_phi_wall(*v)
        sim.step(32)
    got = sim.phi().cpu().numpy()
    ref = oracle_run(spec, phi0, 32 * len(vals), lambda t: vals[min((t + 1) // 32, len(vals) - 1)])
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    say(f"[gpu walls] graph blocks: rel L2 vs oracle {e:.2e}")
    assert e <= 1e-12


def test_set_phi_wall_needs_walls():
    from paper_1603_09577_amd import lbm
    sim = lbm.Lbm(W.spec_nonlinear_2d(16, 12))
    with pytest.raises(lbm.LbmError) as ei:
        sim.set_phi_wall(0.1, 0.2)
    assert ei.value.code == lbm.LBM_E_INVALID
