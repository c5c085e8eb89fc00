"""Grids past the 32-bit offset limit, against the oracle on windows.

A context forms 32-bit byte offsets only while every array it indexes spans
less than 4 GiB (a direction plane of at most 2^29 eight-byte elements);
larger grids take the kernels with 64-bit addressing, and the two-step pass,
which needs the 32-bit forms, is refused.  These cases run D2Q9 (periodic, and
with walls on y) and D3Q19 with walls on z just past that limit, in FP32
offset storage, two steps from Eq. 40.

After two steps a node depends only on the nodes within two lattice links of
it (collision is local, streaming moves one link per step).  So the oracle
runs the same parameters on a window of 5 nodes per axis around each sampled
node, filled from the same phi0 (periodic windows on periodic axes; on a wall
axis the window keeps the real wall where it reaches it, and any wall value
on a side cut out of the interior, which the centre never sees within two
steps), and the window's centre must match the large grid's node.  Samples
include the corners, the faces and the last nodes of the grid.

Bound: max |d| / max |phi| <= 1e-5 over the samples (FP32 storage target).
The window argument itself is checked on the CPU: on small grids, the
oracle's windows reproduce every node of the oracle's full-grid run.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")

STEPS = 2
HALF = STEPS          # window half-width
TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def field_2d(nx, ny):
    """phi0(x, y): a smooth part plus a rough one that differs between
    neighbours (so every population of every node is exercised)."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    smooth = 0.5 + 0.15 * np.cos(2 * np.pi * 3 * y / ny)[:, None] * np.sin(2 * np.pi * 5 * x / nx)[None, :]
    rough = ((7 * np.arange(nx))[None, :] + (13 * np.arange(ny))[:, None]) % 17
    return smooth + 0.01 * rough


def field_3d(nx, ny, nz):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)
    out = np.empty((nz, ny, nx))
    out[:] = (0.4 * np.sin(np.pi * (z + 0.5) / nz))[:, None, None]
    out += (0.1 * np.cos(2 * np.pi * 2 * y / ny))[None, :, None]
    out += (0.05 * np.sin(2 * np.pi * 3 * x / nx))[None, None, :]
    out += 0.002 * (((5 * np.arange(nx))[None, None, :] + (11 * np.arange(ny))[None, :, None]
                     + (3 * np.arange(nz))[:, None, None]) % 13)
    return out


def axis_window(c, n, wall):
    """Indices of the window along one axis and the centre's position in it.
    Periodic: c - HALF .. c + HALF wrapped.  Wall axis: the same span clipped
    into [0, n) and shifted so that it stays 2 * HALF + 1 long."""
    w = 2 * HALF + 1
    if not wall:
        return [(c + d) % n for d in range(-HALF, HALF + 1)], HALF
    lo = min(max(c - HALF, 0), n - w)
    return list(range(lo, lo + w)), c - lo


def window_spec(spec, shape, wall_axis, lo_real, hi_real):
    s = dict(spec)
    s["shape"] = tuple(shape)
    s["precision"] = "f64"
    if wall_axis is not None:
        pw = [list(v) for v in spec["phi_wall"]]
        # a window side cut out of the interior gets an arbitrary wall value
        if not lo_real:
            pw[wall_axis][0] = 0.123
        if not hi_real:
            pw[wall_axis][1] = 0.456
        s["phi_wall"] = pw
    return s


def samples_2d(nx, ny, count=40, seed=11):
    rng = np.random.default_rng(seed)
    pts = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0), (nx // 2, ny - 1),
           (0, ny // 2), (nx - 1, ny // 2), (nx - 1, 1), (1, ny - 2)]
    pts += [(int(rng.integers(nx)), int(rng.integers(ny))) for _ in range(count)]
    return pts


def samples_3d(n, count=30, seed=12):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz - 1), (0, ny - 1, 0), (nx // 2, ny // 2, 0),
           (nx // 2, ny // 2, nz - 1), (3, 5, 1), (nx - 2, ny - 3, nz - 2)]
    pts += [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(count)]
    return pts


def run_large(spec, phi0):
    from paper_1603_09577_amd import lbm
    sim = lbm.Lbm(spec).init(phi0)
    # the 64-bit kernels are the ones running: the two-step pass is refused
    with pytest.raises(lbm.LbmError):
        sim.set_two_step(True)
    sim.step(STEPS)
    phi = sim.phi()
    torch.cuda.synchronize()
    return sim, phi


@pytest.mark.gpu
@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "walls-y"])
def test_d2q9_past_32bit_offsets(walls):
    # 2^29 = 536,870,912 nodes is the first plane of 4 GiB in FP64 terms;
    # nx a multiple of 64 with walls (the row-wave gathers), not without
    nx, ny = (23232, 23200) if walls else (23200, 23200)
    assert nx * ny > 1 << 29
    spec = W.spec_nonlinear_2d(nx, ny, precision="f32")
    wall_axis = None
    if walls:
        spec["bc"] = ["periodic", "abb", "periodic"]
        spec["phi_wall"] = [[0.0, 0.0], [0.3, 0.7], [0.0, 0.0]]
        wall_axis = 1
    say(f"[max size] D2Q9 {nx} x {ny} ({nx * ny} nodes) f32 walls={walls}: building phi0")
    phi0 = field_2d(nx, ny)
    say("[max size] running the GPU")
    sim, phi = run_large(spec, phi0)
    worst, where = 0.0, None
    scale = 0.0
    for (x, y) in samples_2d(nx, ny):
        xs, cx = axis_window(x, nx, False)
        ys, cy = axis_window(y, ny, walls)
        win = phi0[np.ix_(ys, xs)]
        ws = window_spec(spec, (len(xs), len(ys)), wall_axis, ys[0] == 0, ys[-1] == ny - 1)
        o = orc.run(orc.params_from_spec(ws), win, STEPS)[0]
        ov = float(o[cy, cx])
        gv = float(phi[y, x])
        scale = max(scale, abs(ov))
        d = abs(gv - ov)
        if d > worst:
            worst, where = d, (x, y, gv, ov)
    rel = worst / scale
    say(f"[max size] D2Q9 walls={walls}: max |d| / max |phi| = {rel:.2e} at {where}")
    assert np.isfinite(rel) and rel <= TOL
    del sim, phi
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_d3q19_past_32bit_offsets():
    n = (816, 816, 816)
    N = n[0] * n[1] * n[2]
    assert N > 1 << 29
    spec, _, _ = W.d3q19_walls(n, precision="f32")
    spec["phi_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.2, 0.6]]
    say(f"[max size] D3Q19 {n} ({N} nodes) f32 walls on z: building phi0")
    phi0 = field_3d(*n)
    say("[max size] running the GPU")
    sim, phi = run_large(spec, phi0)
    worst, where, scale = 0.0, None, 0.0
    for (x, y, z) in samples_3d(n):
        xs, cx = axis_window(x, n[0], False)
        ys, cy = axis_window(y, n[1], False)
        zs, cz = axis_window(z, n[2], True)
        win = phi0[np.ix_(zs, ys, xs)]
        ws = window_spec(spec, (len(xs), len(ys), len(zs)), 2, zs[0] == 0, zs[-1] == n[2] - 1)
        o = orc.run(orc.params_from_spec(ws), win, STEPS)[0]
        ov = float(o[cz, cy, cx])
        gv = float(phi[z, y, x])
        scale = max(scale, abs(ov))
        d = abs(gv - ov)
        if d > worst:
            worst, where = d, (x, y, z, gv, ov)
    rel = worst / scale
    say(f"[max size] D3Q19: max |d| / max |phi| = {rel:.2e} at {where}")
    assert np.isfinite(rel) and rel <= TOL
    del sim, phi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", ["d2q9-periodic", "d2q9-walls", "d3q19-walls"])
def test_oracle_windows_reproduce_the_full_grid(case):
    """CPU: two steps of the oracle on the full grid against the same two
    steps on the 5-node window of every node (D2Q9) or of sampled nodes
    (D3Q19), including nodes next to the walls and the periodic seams."""
    if case.startswith("d2q9"):
        walls = case.endswith("walls")
        nx, ny = 13, 11
        spec = W.spec_nonlinear_2d(nx, ny, precision="f64")
        wall_axis = None
        if walls:
            spec["bc"] = ["periodic", "abb", "periodic"]
            spec["phi_wall"] = [[0.0, 0.0], [0.3, 0.7], [0.0, 0.0]]
            wall_axis = 1
        phi0 = field_2d(nx, ny)
        full = orc.run(orc.params_from_spec(spec), phi0, STEPS)[0]
        for y in range(ny):
            for x in range(nx):
                xs, cx = axis_window(x, nx, False)
                ys, cy = axis_window(y, ny, walls)
                ws = window_spec(spec, (len(xs), len(ys)), wall_axis, ys[0] == 0, ys[-1] == ny - 1)
                o = orc.run(orc.params_from_spec(ws), phi0[np.ix_(ys, xs)], STEPS)[0]
                assert abs(o[cy, cx] - full[y, x]) <= 1e-14, (x, y, o[cy, cx], full[y, x])
    else:
        n = (9, 8, 10)
        spec, _, _ = W.d3q19_walls(n, precision="f64")
        spec["phi_wall"] = [[0.0, 0.0], [0.0, 0.0], [0.2, 0.6]]
        phi0 = field_3d(*n)
        full = orc.run(orc.params_from_spec(spec), phi0, STEPS)[0]
        pts = samples_3d(n, count=20) + [(x, y, z) for x in (0, 8) for y in (0, 7) for z in (0, 1, 2, 7, 8, 9)]
        for (x, y, z) in pts:
            xs, cx = axis_window(x, n[0], False)
            ys, cy = axis_window(y, n[1], False)
            zs, cz = axis_window(z, n[2], True)
            ws = window_spec(spec, (len(xs), len(ys), len(zs)), 2, zs[0] == 0, zs[-1] == n[2] - 1)
            o = orc.run(orc.params_from_spec(ws), phi0[np.ix_(zs, ys, xs)], STEPS)[0]
            assert abs(o[cz, cy, cx] - full[z, y, x]) <= 1e-14, (x, y, z, o[cz, cy, cx], full[z, y, x])
