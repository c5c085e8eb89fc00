"""The Burgers-Fisher travelling wave (Sec. 3.2, Eq. 46-51) on the GPU:
nonlinear B, the Scheme-A source R = b phi (1 - phi) and anti-bounce-back
walls whose values follow the exact solution step by step (lbm_set_phi_wall).

Against the oracle on the same schedule: FP64 <= 1e-12 (relative L2 and
max |d| / max |phi|), FP32 offsets <= 1e-5; and the GPU's GRE against the
closed form falls at second order (Fig. 4), 2 +- 0.3.
"""
import math
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A_, B_, Y0, LENGTH = 4.0, 1.0, -1.0, 3.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def walls(kappa, dt):
    return lambda t: (float(W.burgers_fisher_wave(Y0, (t + 0.5) * dt, A_, B_, kappa)),
                      float(W.burgers_fisher_wave(Y0 + LENGTH, (t + 0.5) * dt, A_, B_, kappa)))


def setup(n, nx, kappa, precision="f64"):
    spec, dx, dt = W.spec_burgers_fisher(n, nx=nx, a=A_, b=B_, kappa=kappa, length=LENGTH, precision=precision)
    y = Y0 + (np.arange(n) + 0.5) * dx
    wall = walls(kappa, dt)
    # the initial layout is written (and its first gather undone) with these values
    spec["phi_wall"] = [[0, 0], list(wall(0)), [0, 0]]
    phi0 = np.repeat(W.burgers_fisher_wave(y, 0.0, A_, B_, kappa)[:, None], nx, axis=1)
    return spec, phi0, y, dt, wall


def gpu_wave(spec, phi0, nst, wall):
    """Pull form: phi_w(t), used by the streaming of step t, is set right after
    the sweep of step t."""
    from paper_1603_09577_amd import lbm
    sim = lbm.Lbm(spec).init(phi0)
    for t in range(nst):
        sim.step(1)
        sim.set_phi_wall(*wall(t))
    return sim.phi().cpu().numpy()


def oracle_wave(spec, phi0, nst, wall):
    p = orc.params_from_spec(dict(spec, precision="f64"))
    f, pp = orc.init(p, phi0)
    for t in range(nst):
        p.phi_wall[1][0], p.phi_wall[1][1] = wall(t)
        orc.step(p, f, pp)
    return orc.phi(p, f)


@pytest.mark.parametrize("nx,prec,tol", [(2, "f64", 1e-12), (64, "f64", 1e-12), (64, "f32", 1e-5)])
def test_wave_against_oracle(nx, prec, tol):
    n, kappa = 96, 0.1
    spec, phi0, y, dt, wall = setup(n, nx, kappa, prec)
    nst = int(round(0.5 / dt))
    say(f"[gpu burgers-fisher] {nx}x{n} {prec} {nst} steps")
    got = gpu_wave(spec, phi0, nst, wall)
    ref = oracle_wave(spec, phi0, nst, wall)
    e2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    ep = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"    rel L2 {e2:.2e}, max |d| / max |phi| {ep:.2e}")
    assert e2 <= tol and ep <= tol


def test_wave_second_order_on_gpu():
    kappa = 0.1
    gres = []
    for n in (96, 192, 384):
        spec, phi0, y, dt, wall = setup(n, 64, kappa)
        nst = int(round(0.5 / dt))
        say(f"[gpu burgers-fisher] order: 64x{n}, {nst} steps")
        got = gpu_wave(spec, phi0, nst, wall)
        ex = np.repeat(W.burgers_fisher_wave(y, nst * dt, A_, B_, kappa)[:, None], 64, axis=1)
        gres.append(float(np.abs(got - ex).sum() / np.abs(ex).sum()))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(2)]
    say(f"    GRE {gres}, orders {order}")
    assert all(1.7 <= o <= 2.3 for o in order), (gres, order)
