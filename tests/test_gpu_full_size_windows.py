"""The full-size D3Q19 workload (256^3 with walls) in the launch configuration
the benchmark times (autotuned: two steps per pass, XCD-aware order), against
the oracle on windows, for more steps than a full-grid oracle run allows.

After s steps a node depends only on the nodes within s lattice links of it,
so the oracle runs the same parameters on the window of 2s + 1 nodes per
axis around a sampled node (periodic windows on x and y; on z the window
keeps the real wall where it reaches it and any wall value on a side cut out
of the interior, which the centre cannot see within s steps; the CPU test in
test_gpu_max_size.py checks this argument against full-grid oracle runs), and
the window's centre must match the GPU's node.

Bounds: max |d| / max |phi| over the samples <= 1e-12 (FP64) and 1e-5 (FP32).
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STEPS = 24          # six pairs of two-step passes


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def axis_window(c, n, wall, half):
    w = 2 * half + 1
    if not wall:
        return [(c + d) % n for d in range(-half, half + 1)], half
    lo = min(max(c - half, 0), n - w)
    return list(range(lo, lo + w)), c - lo


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_d3q19_full_size_tuned_windows(prec, tol):
    from paper_1603_09577_amd import lbm
    spec, phi0, _ = W.d3q19_walls(precision=prec)
    n = spec["shape"]
    say(f"[full size] D3Q19 {n} {prec}: tuned run of {STEPS} steps")
    sim = lbm.Lbm(spec).init(phi0)
    rep = sim.tune(reps=5).splitlines()[-1]
    say(f"    tuner: {rep}")
    sim.step(STEPS)
    phi = sim.phi().cpu().numpy()
    rng = np.random.default_rng(17)
    pts = [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (61, 62, 1), (62, 13, n[2] - 2), (128, 200, 27)]
    pts += [tuple(int(rng.integers(m)) for m in n) for _ in range(5)]
    # and where the field is large: the highest node of phi0 and nodes beside it
    zm, ym, xm = np.unravel_index(int(np.argmax(phi0)), phi0.shape)
    pts += [(int(xm), int(ym), int(zm)), (int(xm) + 3, int(ym) - 2, int(zm)), (int(xm), int(ym) + 5, max(int(zm) - 4, 0))]
    pts = [(x % n[0], y % n[1], z) for (x, y, z) in pts]
    worst, where, scale = 0.0, None, 0.0
    for (x, y, z) in pts:
        xs, cx = axis_window(x, n[0], False, STEPS)
        ys, cy = axis_window(y, n[1], False, STEPS)
        zs, cz = axis_window(z, n[2], True, STEPS)
        ws = dict(spec, shape=(len(xs), len(ys), len(zs)), precision="f64")
        pw = [list(v) for v in spec["phi_wall"]]
        if zs[0] != 0:
            pw[2][0] = 0.123
        if zs[-1] != n[2] - 1:
            pw[2][1] = 0.456
        ws["phi_wall"] = pw
        o = orc.run(orc.params_from_spec(ws), phi0[np.ix_(zs, ys, xs)], STEPS)[0]
        ov, gv = float(o[cz, cy, cx]), float(phi[z, y, x])
        scale = max(scale, abs(ov))
        if abs(gv - ov) > worst:
            worst, where = abs(gv - ov), (x, y, z, gv, ov)
    rel = worst / scale
    say(f"    max |d| / max |phi| = {rel:.2e} at {where}")
    assert np.isfinite(rel) and rel <= tol
