"""GPU forward sweep against the CPU oracle, element by element.

Every case starts both sides from the same seeded phi0 (workloads module) and
compares phi after a number of steps, by relative L2 over all nodes and by the
largest pointwise difference relative to the largest |phi| of the oracle
(so that a wrong value at a few nodes, a wall row or the last column of a
ragged tile, cannot hide in the norm of a large grid), both against:
    FP64 storage    <= 1e-12   (the target stated for the FP64 path)
    FP32 offsets    <= 1e-5    (the target stated for FP32 storage)
    FP16 offsets    reported, loose sanity bound only.
The node with the largest difference is printed with every comparison.
Sizes are chosen to span several 256-node workgroups with a ragged tail;
the full-size cases run a few steps at the benchmark's configuration.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lbm():
    from paper_1603_09577_amd import lbm
    return lbm


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """max |a - b| / max |b|, and the index of the worst node."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b)
    i = np.unravel_index(int(np.argmax(d)), d.shape)
    return float(d[i] / np.abs(b).max()), tuple(int(v) for v in i)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(spec, phi0, snapshots, flags=0):
    lbm = _lbm()
    sim = lbm.Lbm(spec, flags=flags).init(phi0)
    out = {}
    t = 0
    for s in sorted(snapshots):
        sim.step(s - t)
        t = s
        out[s] = sim.phi().cpu().numpy()
    torch.cuda.synchronize()
    return out


def oracle_run(spec, phi0, snapshots):
    p = orc.params_from_spec(spec)
    last = max(snapshots)
    _, snaps = orc.run(p, phi0, last, snapshots=tuple(snapshots))
    return snaps


def compare(spec, phi0, snapshots, tol, flags=0, name=""):
    say(f"[gpu parity] {name} shape={spec['shape']} prec={spec.get('precision')} flags={flags} steps={snapshots}")
    g = gpu_run(spec, phi0, snapshots, flags)
    o = oracle_run(spec, phi0, snapshots)
    errs = {s: rel_l2(g[s], o[s]) for s in snapshots}
    pts = {s: max_rel(g[s], o[s]) for s in snapshots}
    say(f"    rel L2 {errs}")
    say("    max |d| / max |phi| (worst node) " + ", ".join(f"{s}: {v:.2e} at {i}" for s, (v, i) in pts.items()))
    for s in snapshots:
        assert np.isfinite(g[s]).all(), (name, s)
        assert errs[s] <= tol, (name, s, errs[s])
        assert pts[s][0] <= tol, (name, s, pts[s])
    return errs


# ---------------------------------------------------------------------------
# D2Q9
# ---------------------------------------------------------------------------

def test_c1_full_fp64_moment_path():
    """Linear Gaussian hill, 64 x 64, 1000 steps, s1 = s2 = 1.2 (moment path)."""
    spec, phi0, T = W.hill_linear_64()
    compare(spec, phi0, (1, 250, 500, T), 1e-12, name="hill_linear_64")


@pytest.mark.parametrize("flags", [0, 1])
def test_nonlinear_small_fp64(flags):
    """Nonlinear B, K(phi), Scheme-A source on a ragged 72 x 41 grid; both the
    equal-rate path (flags = 0) and the forced moment path (flags = 1)."""
    spec = W.spec_nonlinear_2d(72, 41)
    phi0 = W.noise_field((41, 72), 12)
    compare(spec, phi0, (1, 10, 100, 400), 1e-12, flags=flags, name="nonlinear-2d")


def test_general_rates_anisotropic_fp64():
    """Unequal non-flux rates, full K0, nonlinear D and d != 1 (moment path)."""
    spec = W.spec_nonlinear_2d(50, 37)
    spec["s"] = [0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05]
    spec["d"] = 0.8
    spec["dpoly"] = [0.05, 0.9, 0.1]
    phi0 = W.noise_field((37, 50), 13)
    compare(spec, phi0, (1, 50, 300), 1e-12, name="general-rates")


def test_channel_walls_fp64():
    """D2Q9 anti-bounce-back walls on y with different wall values."""
    spec = W.spec_nonlinear_2d(40, 33, source=True)
    spec["bc"] = ["periodic", "abb", "periodic"]
    spec["phi_wall"] = [[0, 0], [0.3, 0.8], [0, 0]]
    phi0 = W.noise_field((33, 40), 14)
    compare(spec, phi0, (1, 20, 200), 1e-12, name="channel")
    spec["s"] = [0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05]
    compare(spec, phi0, (1, 20, 200), 1e-12, name="channel-general-rates")


@pytest.mark.parametrize("walls,prec,tol", [(False, "f64", 1e-12), (True, "f64", 1e-12), (True, "f32", 1e-5)])
def test_row_wave_sweeps(walls, prec, tol):
    """Widths that are multiples of 64 put every wave within one grid row; with
    walls the one-sweep kernel then takes its row-wave gathers (scalar row
    offsets, per-lane columns).  The periodic case (two steps per pass off)
    runs the general gathers on the same grid."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(128, 11, source=True, precision=prec)
    if walls:
        spec["bc"] = ["periodic", "abb", "periodic"]
        spec["phi_wall"] = [[0, 0], [0.3, 0.8], [0, 0]]
    phi0 = W.noise_field((11, 128), 15)
    say(f"[gpu parity] row waves 128x11 walls={walls} {prec}")
    sim = lbm.Lbm(spec).init(phi0)
    if not walls:
        sim.set_two_step(False)
    sim.step(40)
    ref = oracle_run(dict(spec, precision="f64"), phi0, (40,))[40]
    got = sim.phi().cpu().numpy()
    err, (pt, at) = rel_l2(got, ref), max_rel(got, ref)
    say(f"    rel L2 {err:.2e}, max |d| / max |phi| {pt:.2e} at {at}")
    assert err <= tol and pt <= tol


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f16", 2e-2)])
def test_nonlinear_reduced_storage(prec, tol):
    """FP32 / FP16 offset storage against the FP64 oracle."""
    spec = W.spec_nonlinear_2d(96, 80, precision=prec)
    phi0 = W.noise_field((80, 96), 15)
    compare(spec, phi0, (1, 10, 100, 1000), tol, name=f"nonlinear-{prec}")


def test_c2_full_size_fp64_and_fp32():
    """The benchmark configuration (1024 x 1024) for a few steps: FP64 <= 1e-12
    and FP32 offsets <= 1e-5 against the oracle at full size."""
    spec, phi0, _ = W.nonlinear_2d(1024)
    compare(spec, phi0, (1, 4), 1e-12, name="nonlinear2d-1024-f64")
    spec32, _, _ = W.nonlinear_2d(1024, precision="f32")
    compare(spec32, phi0, (1, 4), 1e-5, name="nonlinear2d-1024-f32")


# ---------------------------------------------------------------------------
# D3Q19
# ---------------------------------------------------------------------------

def test_d3q19_walls_fp64():
    """D3Q19 wall-bounded anisotropic physics on a ragged 21 x 18 x 26 grid with z walls (equal rates)."""
    spec, phi0, _ = W.d3q19_walls((21, 18, 26))
    compare(spec, phi0, (1, 30, 150), 1e-12, name="d3q19-walls")


def test_d3q19_everything_fp64():
    """D3Q19 with nonlinear B, K(phi), D, source, nonzero wall values and
    unequal rates (moment path), and the same with forced moment path on
    equal rates."""
    spec = W.spec_d3q19_aniso((13, 11, 17), phi_wall=0.4)
    spec["b"] = [[0.0, 0.02, 0.03], [0.0, -0.01, 0.02], [0.0, 0.01, -0.02]]
    spec["kpoly"] = [1.0, 0.0, 0.5]
    spec["rpoly"] = [0.0, 0.002, -0.002]
    spec["dpoly"] = [0.02, 0.95]
    spec["phi_wall"] = [[0, 0], [0, 0], [0.2, 0.6]]
    rng = np.random.default_rng(16)
    phi0 = 0.4 + 0.1 * rng.uniform(-1, 1, (17, 11, 13))
    compare(spec, phi0, (1, 40), 1e-12, flags=1, name="d3q19-moment-equal")
    spec["s"] = [0.0] + [1.0 + 0.04 * i for i in range(18)]
    compare(spec, phi0, (1, 40), 1e-12, name="d3q19-general")


def test_d3q19_fp32():
    spec, phi0, _ = W.d3q19_walls((32, 24, 40), precision="f32")
    compare(spec, phi0, (1, 50, 200), 1e-5, name="d3q19-f32")


def test_c3_full_size_two_steps():
    """The D3Q19 benchmark grid (256^3, walls) for two steps, FP64 and FP32."""
    spec, phi0, _ = W.d3q19_walls()
    compare(spec, phi0, (2,), 1e-12, name="d3q19-256-f64")
    spec32, _, _ = W.d3q19_walls(precision="f32")
    compare(spec32, phi0, (2,), 1e-5, name="d3q19-256-f32")


# ---------------------------------------------------------------------------
# properties on the GPU
# ---------------------------------------------------------------------------

def test_conservation_reduction_fp64():
    """Periodic, R = 0: the FP64 reduction of sum phi is conserved."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(200, 130, source=False)
    phi0 = W.noise_field((130, 200), 17)
    say("[gpu] conservation 200x130")
    sim = lbm.Lbm(spec).init(phi0)
    s0 = sim.reduce(sim.phi())["sum"]
    sim.step(500)
    r = sim.reduce(sim.phi())
    assert r["nonfinite"] == 0
    assert abs(r["sum"] - s0) <= 1e-13 * abs(s0)
    assert abs(s0 - phi0.sum()) <= 1e-13 * abs(s0)


def test_reduce_async_equals_reduce():
    """lbm_reduce_async writes the 8 values of lbm_reduce, bit for bit, to
    device memory; several in flight on the stream before one read, with and
    without a reference field; values checked against numpy in FP64."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(200, 130)
    phi0 = W.noise_field((130, 200), 18)
    say("[gpu] reduce_async 200x130")
    sim = lbm.Lbm(spec).init(phi0)
    sim.step(7)
    phi = sim.phi()
    ref = torch.tensor(W.noise_field((130, 200), 19), dtype=torch.float64, device="cuda")
    outs = [sim.reduce_async(phi), sim.reduce_async(phi, ref)]
    sim.step(3)
    phi2 = sim.phi()
    outs.append(sim.reduce_async(phi2, ref))
    torch.cuda.synchronize()
    keys = ("sum", "sumsq", "sum_d2", "sum_ref2", "min", "max", "nonfinite", "sum_absd")
    for o, (p, r) in zip(outs, ((phi, None), (phi, ref), (phi2, ref))):
        want = sim.reduce(p, r)
        got = o.cpu().numpy()
        assert [got[i] for i in range(8)] == [want[k] for k in keys]
    p, r = phi2.cpu().numpy(), ref.cpu().numpy()
    got = outs[2].cpu().numpy()
    assert abs(got[0] - p.sum()) <= 1e-13 * abs(p.sum())
    assert abs(got[2] - ((p - r) ** 2).sum()) <= 1e-12 * ((p - r) ** 2).sum()
    assert got[4] == p.min() and got[5] == p.max() and got[6] == 0


@pytest.mark.parametrize("case", ["periodic-f32", "walls-f64", "d3q19-f32", "d3q19-f16"])
def test_reduce_state_equals_reduce_of_phi(case):
    """lbm_reduce_state forms phi from the stored populations inside the
    reduction; its 8 values equal, bit for bit, those of lbm_reduce over the
    field lbm_get_phi writes, with and without a reference field."""
    lbm = _lbm()
    if case == "periodic-f32":
        spec = W.spec_nonlinear_2d(200, 130, precision="f32")
    elif case == "walls-f64":
        spec = dict(W.spec_nonlinear_2d(130, 70), bc=["periodic", "abb", "periodic"],
                    phi_wall=[[0, 0], [0.3, 0.8], [0, 0]])
    else:
        spec = W.d3q19_walls((20, 18, 22), precision=case[-3:])[0]
    sim = lbm.Lbm(spec)
    phi0 = W.noise_field(tuple(sim.shape), 20)
    say(f"[gpu] reduce_state {case} {sim.shape}")
    sim.init(phi0)
    sim.step(9)
    ref = torch.tensor(W.noise_field(tuple(sim.shape), 21), dtype=torch.float64, device="cuda")
    keys = ("sum", "sumsq", "sum_d2", "sum_ref2", "min", "max", "nonfinite", "sum_absd")
    for r in (None, ref):
        got = sim.reduce_state(r).cpu().numpy()
        want = sim.reduce(sim.phi(), r)
        assert [got[i] for i in range(8)] == [want[k] for k in keys], (case, r is None)


def test_every_node_written():
    """Poison the destination with NaN: one sweep must overwrite every value."""
    lbm = _lbm()
    for spec, phi0 in ((W.spec_nonlinear_2d(77, 29), W.noise_field((29, 77), 18)),
                       (W.d3q19_walls((9, 7, 11))[0], W.d3q19_walls((9, 7, 11))[1])):
        say(f"[gpu] poison {spec['shape']}")
        sim = lbm.Lbm(spec).init(phi0)
        view = sim.storage_view(sim.f[1])
        view.fill_(float("nan"))
        sim.step(1)
        assert torch.isfinite(view).all().item()
        assert torch.isfinite(sim.phi()).all().item()


def test_divergence_detected():
    """An unstable BGK setting (Sec. 3.6, kappa = 1e-4) trips the NaN check."""
    lbm = _lbm()
    n, dx = 64, 2.0 / 400
    kl = 1e-4 * dx / dx ** 2
    sj = 1.0 / (3 * kl + 0.5)
    spec = dict(lattice=9, shape=(n, n), bc=["periodic"] * 3, scheme="A", d=1.0, s=[sj] * 9,
                b=[[0.0, 0.1], [0.0, 0.1]], dpoly=[0, 1], dten=[[1, 1, 0], [1, 2, 0], [0, 0, 1]],
                k0=(kl * np.eye(3)).tolist(), kpoly=[1.0], rpoly=[])
    say("[gpu] divergence check")
    sim = lbm.Lbm(spec).init(W.gaussian_hill(n, 2.0))
    sim.set_check(50)
    with pytest.raises(lbm.LbmError) as e:
        sim.step(3000)
    assert e.value.code == lbm.LBM_E_DIVERGED


def test_divergence_check_keeps_two_step_passes():
    """With the divergence check on, the steps between checks still run as
    two-step passes: the result is the same bit for bit as without the check
    (which runs graphs of passes), for check intervals that are and are not
    multiples of 4, and an unstable run is still caught."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(130, 50, precision="f32")
    phi0 = W.noise_field((50, 130), 41)
    say("[gpu] divergence check with two-step passes")
    ref = lbm.Lbm(spec).init(phi0)
    ref.step(103)
    for every in (8, 10, 7):
        sim = lbm.Lbm(spec).init(phi0)
        sim.set_check(every)
        sim.step(51)
        sim.step(52)
        assert torch.equal(sim.phi(), ref.phi()), every
        wa, _ = sim.current()
        wb, _ = ref.current()
        assert wa == wb


def test_graph_replay_identical_to_direct_launches():
    """lbm_step replays captured 32-sweep graphs; the result is bit-identical
    to launching every sweep directly."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(96, 70, precision="f32")
    phi0 = W.noise_field((70, 96), 19)
    say("[gpu] graph replay vs direct")
    a = lbm.Lbm(spec).init(phi0)
    a.step(100)
    b = lbm.Lbm(spec, flags=lbm.FLAG_NO_GRAPH).init(phi0)
    b.step(100)
    assert torch.equal(a.phi(), b.phi())
    c = lbm.Lbm(spec, flags=lbm.FLAG_NO_XCD_REMAP).init(phi0)
    c.step(100)
    assert torch.equal(a.phi(), c.phi())


def test_launch_variants_identical():
    """Non-temporal accesses, chunked workgroups, the XCD block order and the
    autotuned shape change only how the sweep is launched: results are
    bit-identical."""
    lbm = _lbm()
    for spec, phi0 in ((W.spec_nonlinear_2d(150, 90, precision="f32"), W.noise_field((90, 150), 20)),
                       (W.d3q19_walls((20, 18, 22))[0], W.d3q19_walls((20, 18, 22))[1])):
        say(f"[gpu] launch variants {spec['shape']}")
        ref = lbm.Lbm(spec).init(phi0)
        ref.step(70)
        want = ref.phi()
        for nt, chunk, fl in ((1, 1, 0), (0, 3, 0), (1, 5, 0), (0, 3, lbm.FLAG_NO_XCD_REMAP),
                              (1, 2, lbm.FLAG_NO_XCD_REMAP)):
            s = lbm.Lbm(spec, flags=fl).init(phi0)
            s.set_nontemporal(nt)
            s.set_chunk(chunk)
            s.step(70)
            assert torch.equal(s.phi(), want), (nt, chunk, fl)
        for remap in (0, 1):
            s = lbm.Lbm(spec).init(phi0)
            s.set_remap(remap)
            s.step(70)
            assert torch.equal(s.phi(), want), remap
        s = lbm.Lbm(spec).init(phi0)
        s.tune(reps=2)
        s.step(70)
        assert torch.equal(s.phi(), want)


@pytest.mark.parametrize("nx,ny,prec,source,shape", [(100, 37, "f32", True, 0), (190, 23, "f64", True, 0),
                                                     (130, 50, "f16", True, 0), (64, 16, "f32", False, 0),
                                                     (257, 91, "f64", False, 0), (100, 37, "f32", True, 1),
                                                     (131, 29, "f32", True, 2), (130, 50, "f16", True, 3),
                                                     (64, 16, "f16", False, 1), (190, 23, "f64", True, 1),
                                                     (70, 16, "f32", True, 3), (130, 29, "f64", True, 2),
                                                     (40, 30, "f32", True, 1), (33, 7, "f64", True, 0),
                                                     (20, 5, "f16", True, 3), (61, 13, "f64", False, 2),
                                                     (3, 2, "f32", True, 0)])
def test_two_step_passes_bit_identical(nx, ny, prec, source, shape):
    """Two time steps per pass (LDS tiles of 62 x 14, 10 or 6 nodes with a
    one-node halo, 4, 6 or 8 waves per workgroup) against single sweeps: the same arithmetic on the same
    inputs, so phi, the stored state and the phi history agree bit for bit,
    across graph replays, passes in pairs and single-sweep remainders; and the
    result matches the oracle."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(nx, ny, source=source, precision=prec)
    phi0 = W.noise_field((ny, nx), 71)
    say(f"[gpu] two-step passes {nx}x{ny} {prec} source={source} shape={shape}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    b.set_two_step(True, shape)
    t = 0
    for s in (4, 8, 37, 70):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
        if source:   # the N history values (the buffer tail is padding)
            hdt = torch.float64 if prec == "f64" else torch.float32
            assert torch.equal(a.p.view(hdt)[: a.N], b.p.view(hdt)[: b.N]), s
    if prec == "f64":
        ref = oracle_run(spec, phi0, (70,))[70]
        got = b.phi().cpu().numpy()
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("nx,ny,prec,shape", [(100, 37, "f32", 0), (190, 23, "f64", 0), (130, 50, "f16", 0),
                                               (131, 29, "f32", 1), (61, 13, "f64", 1), (20, 5, "f16", 3),
                                               (3, 2, "f32", 2)])
def test_two_step_passes_scheme_b_bit_identical(nx, ny, prec, shape):
    """Scheme B with R(phi) (Eq. 35 solved at every node of both phases) in
    two-step passes against single sweeps of the same 3-term kernel: phi and
    the stored state agree bit for bit; no second history is asked for; the
    FP64 result matches the oracle."""
    lbm = _lbm()
    spec = dict(W.spec_nonlinear_2d(nx, ny, precision=prec), scheme="B")
    phi0 = W.noise_field((ny, nx), 73)
    say(f"[gpu] two-step passes scheme B {nx}x{ny} {prec} shape={shape}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    assert b.p2 is None
    b.set_two_step(True, shape)
    t = 0
    for s in (4, 8, 37, 70):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
    if prec == "f64":
        ref = oracle_run(spec, phi0, (70,))[70]
        got = b.phi().cpu().numpy()
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("n,prec,wall,shape", [((20, 18, 22), "f32", True, 0), ((20, 18, 22), "f64", True, 0),
                                                ((70, 13, 9), "f32", False, 1), ((33, 7, 11), "f64", False, 1),
                                                ((65, 9, 17), "f32", True, 2), ((9, 5, 4), "f16", True, 0),
                                                ((3, 2, 2), "f32", True, 1), ((1, 1, 3), "f64", False, 0),
                                                ((64, 30, 40), "f64", True, 0), ((130, 37, 21), "f32", True, 0),
                                                ((40, 20, 30), "f16", False, 2), ((5, 4, 1), "f64", True, 0),
                                                ((7, 3, 2), "f32", True, 1), ((66, 15, 1), "f32", False, 0)])
def test_two_step_passes_d3q19_bit_identical(n, prec, wall, shape):
    """D3Q19 two steps per pass (columns of 62 x 14, 6 or 2 nodes marching up
    chunks of z planes through an LDS ring) against single sweeps: phi and the
    stored state agree bit for bit after even and odd step counts, with and
    without walls on z, on grids narrower and lower than a tile; the FP64
    result matches the oracle."""
    lbm = _lbm()
    spec, _, _ = W.d3q19_walls(n, precision=prec)
    if not wall:
        spec["bc"] = ["periodic"] * 3
    spec["phi_wall"] = [[0, 0], [0, 0], [0.3, 0.6]] if wall else spec["phi_wall"]
    phi0 = W.gaussians_3d(n, 21)
    say(f"[gpu] two-step passes d3q19 {n} {prec} walls={wall} shape={shape}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    b.set_two_step(True, shape)
    t = 0
    for s in (4, 8, 37, 70):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
    if prec == "f64":
        ref = oracle_run(spec, phi0, (70,))[70]
        got = b.phi().cpu().numpy()
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("n,prec,wall,shape", [((20, 18, 22), "f64", True, 0), ((33, 7, 11), "f32", False, 1),
                                                ((70, 16, 9), "f32", True, 0), ((9, 5, 4), "f16", True, 0),
                                                ((5, 4, 1), "f64", True, 1)])
def test_two_step_passes_d3q19_scheme_b_bit_identical(n, prec, wall, shape):
    """D3Q19 in Scheme B with R(phi) of degree 2 (Eq. 35 solved per node):
    Scheme B keeps no phi history, so the two-step pass applies, and it
    matches single sweeps bit for bit; FP64 against the oracle."""
    lbm = _lbm()
    spec, _, _ = W.d3q19_walls(n, precision=prec)
    spec = dict(spec, scheme="B", rpoly=[0.002, 0.01, -0.01])
    if not wall:
        spec["bc"] = ["periodic"] * 3
    spec["phi_wall"] = [[0, 0], [0, 0], [0.3, 0.6]] if wall else spec["phi_wall"]
    phi0 = W.gaussians_3d(n, 23)
    say(f"[gpu] two-step passes d3q19 scheme B {n} {prec} walls={wall} shape={shape}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    b.set_two_step(True, shape)
    t = 0
    for s in (4, 9, 40):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
    if prec == "f64":
        ref = oracle_run(spec, phi0, (40,))[40]
        got = b.phi().cpu().numpy()
        say(f"    vs oracle: rel L2 {rel_l2(got, ref):.2e}, max {max_rel(got, ref)}")
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("n,prec,wall,shape", [((20, 18, 22), "f64", True, 0), ((33, 7, 11), "f32", False, 1),
                                                ((70, 16, 9), "f32", True, 0), ((9, 5, 4), "f16", True, 0),
                                                ((5, 4, 1), "f64", True, 1), ((65, 9, 17), "f32", True, 2)])
def test_two_step_passes_d3q19_scheme_a_source_bit_identical(n, prec, wall, shape):
    """D3Q19 with a Scheme-A source R(phi) (Eq. 9 with the phi history): the
    pass reads the history of its nodes from one buffer, keeps phi(t) in LDS
    for the second step and writes phi(t + 1) to the caller's second history
    buffer; state, history and phi match single sweeps bit for bit; FP64
    against the oracle."""
    lbm = _lbm()
    spec, _, _ = W.d3q19_walls(n, precision=prec)
    spec = dict(spec, rpoly=[0.002, 0.01, -0.01], kpoly=[1.0, 0.0, 0.5])
    if not wall:
        spec["bc"] = ["periodic"] * 3
    spec["phi_wall"] = [[0, 0], [0, 0], [0.3, 0.6]] if wall else spec["phi_wall"]
    phi0 = W.gaussians_3d(n, 24)
    say(f"[gpu] two-step passes d3q19 scheme A source {n} {prec} walls={wall} shape={shape}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    assert b.p2 is not None
    b.set_two_step(True, shape)
    t = 0
    for s in (4, 9, 40):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
        nb = a.N * (8 if prec == "f64" else 4)   # the history proper, not the buffer's padding
        assert torch.equal(a.p[:nb], b.p[:nb]), s
    if prec == "f64":
        ref = oracle_run(spec, phi0, (40,))[40]
        got = b.phi().cpu().numpy()
        say(f"    vs oracle: rel L2 {rel_l2(got, ref):.2e}, max {max_rel(got, ref)}")
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("nx,ny,prec,source,shape", [(100, 37, "f64", "A", 0), (100, 37, "f32", "A", 1),
                                                      (130, 50, "f16", "none", 0), (61, 13, "f64", "B", 1),
                                                      (131, 29, "f32", "B", 2), (64, 64, "f32", "none", 3),
                                                      (3, 2, "f32", "A", 1), (70, 1, "f64", "A", 0),
                                                      (190, 23, "f64", "none", 2)])
def test_two_step_passes_walls_bit_identical(nx, ny, prec, source, shape):
    """D2Q9 with anti-bounce-back walls on y (fixed wall values) in two steps
    per pass: phase 1 skips the rows beyond the walls and both phases take the
    one-sweep wall form, so phi, the state and the history match single
    sweeps bit for bit (Scheme A with its history, Scheme B, no source; tile
    shapes; grids lower than a tile and a single row); FP64 against the
    oracle."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(nx, ny, precision=prec, source=(source != "none"))
    spec = dict(spec, bc=["periodic", "abb", "periodic"], phi_wall=[[0, 0], [0.3, 0.7], [0, 0]])
    if source == "B":
        spec["scheme"] = "B"
    phi0 = W.noise_field((ny, nx), 31)
    say(f"[gpu] two-step passes with walls {nx}x{ny} {prec} source={source} shape={shape}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    b.set_two_step(True, shape)
    t = 0
    for s in (4, 9, 40):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
        if source == "A":
            nb = a.N * (8 if prec == "f64" else 4)
            assert torch.equal(a.p[:nb], b.p[:nb]), s
    if prec == "f64":
        ref = oracle_run(spec, phi0, (40,))[40]
        got = b.phi().cpu().numpy()
        say(f"    vs oracle: rel L2 {rel_l2(got, ref):.2e}, max {max_rel(got, ref)}")
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("nx,ny,prec,source,walls", [(100, 37, "f64", "A", False), (100, 37, "f32", "A", True),
                                                      (130, 50, "f16", "none", False), (61, 13, "f64", "B", True),
                                                      (131, 29, "f32", "B", False), (3, 2, "f64", "A", False),
                                                      (70, 1, "f32", "none", True)])
def test_two_step_passes_unequal_rates_bit_identical(nx, ny, prec, source, walls):
    """Unequal non-flux rates, d != 1 and a nonlinear D (the moment-space
    collision of Eq. 2 with S of Eq. 17) in two steps per pass: bit-identical
    to single sweeps (state, history, phi), periodic or with walls on y, with
    no source, Scheme A or Scheme B; FP64 against the oracle."""
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(nx, ny, precision=prec, source=(source != "none"))
    spec["s"] = [0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05]
    spec["d"] = 0.8
    spec["dpoly"] = [0.05, 0.9, 0.1]
    if walls:
        spec = dict(spec, bc=["periodic", "abb", "periodic"], phi_wall=[[0, 0], [0.3, 0.7], [0, 0]])
    if source == "B":
        spec["scheme"] = "B"
    phi0 = W.noise_field((ny, nx), 33)
    say(f"[gpu] two-step passes, unequal rates {nx}x{ny} {prec} source={source} walls={walls}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    b.set_two_step(True)
    t = 0
    for s in (4, 9, 40):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
        if source == "A":
            nb = a.N * (8 if prec == "f64" else 4)
            assert torch.equal(a.p[:nb], b.p[:nb]), s
    with pytest.raises(lbm.LbmError):
        b.set_two_step(True, 1)   # the moment-space collision has the default tile shape only
    if prec == "f64":
        ref = oracle_run(spec, phi0, (40,))[40]
        got = b.phi().cpu().numpy()
        say(f"    vs oracle: rel L2 {rel_l2(got, ref):.2e}, max {max_rel(got, ref)}")
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


@pytest.mark.parametrize("n,prec,wall,source", [((20, 18, 22), "f64", True, "A"), ((33, 7, 11), "f32", False, "none"),
                                                 ((70, 16, 9), "f32", True, "B"), ((9, 5, 4), "f16", True, "none"),
                                                 ((5, 4, 1), "f64", True, "B"), ((65, 9, 17), "f32", True, "A")])
def test_two_step_passes_d3q19_unequal_rates_bit_identical(n, prec, wall, source):
    """D3Q19 with unequal non-flux rates (the moment-space collision in the
    d'Humieres basis, whose rate slots the paper does not fix) in two steps per pass, default tile shape:
    bit-identical to single sweeps (state, history, phi), with no source,
    Scheme A or Scheme B; FP64 against the oracle."""
    lbm = _lbm()
    spec, _, _ = W.d3q19_walls(n, precision=prec)
    spec = dict(spec, s=[0.0] + [1.0 + 0.03 * ((7 * i) % 11) for i in range(1, 19)])
    if source != "none":
        spec = dict(spec, rpoly=[0.002, 0.01, -0.01], kpoly=[1.0, 0.0, 0.5], scheme=source)
    if not wall:
        spec["bc"] = ["periodic"] * 3
    spec["phi_wall"] = [[0, 0], [0, 0], [0.3, 0.6]] if wall else spec["phi_wall"]
    phi0 = W.gaussians_3d(n, 25)
    say(f"[gpu] two-step passes d3q19 unequal rates {n} {prec} walls={wall} source={source}")
    a = lbm.Lbm(spec).init(phi0)
    a.set_two_step(False)
    b = lbm.Lbm(spec).init(phi0)
    b.set_two_step(True)
    t = 0
    for s in (4, 9, 30):
        a.step(s - t)
        b.step(s - t)
        t = s
        assert torch.equal(a.phi(), b.phi()), s
        wa, _ = a.current()
        wb, _ = b.current()
        assert wa == wb
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb])), s
        if source == "A":
            nb = a.N * (8 if prec == "f64" else 4)
            assert torch.equal(a.p[:nb], b.p[:nb]), s
    with pytest.raises(lbm.LbmError):
        b.set_two_step(True, 1)   # the moment-space collision has the default tile shape only
    if prec == "f64":
        ref = oracle_run(spec, phi0, (30,))[30]
        got = b.phi().cpu().numpy()
        say(f"    vs oracle: rel L2 {rel_l2(got, ref):.2e}, max {max_rel(got, ref)}")
        assert rel_l2(got, ref) <= 1e-12 and max_rel(got, ref)[0] <= 1e-12


def test_two_step_passes_f16_walls_source_with_recentring():
    """FP16 offsets with a Scheme-A source re-centre every 256 steps; between
    walls, with unequal rates and with equal ones, 600 steps in two-step
    passes (re-centred at the same steps) match single sweeps bit for bit."""
    lbm = _lbm()
    for rates in (None, [0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05]):
        spec = W.spec_nonlinear_2d(100, 37, precision="f16")
        spec = dict(spec, bc=["periodic", "abb", "periodic"], phi_wall=[[0, 0], [0.3, 0.7], [0, 0]])
        if rates:
            spec["s"] = rates
        phi0 = W.noise_field((37, 100), 35)
        say(f"[gpu] f16 walls source re-centring, unequal rates={bool(rates)}")
        a = lbm.Lbm(spec).init(phi0)
        a.set_two_step(False)
        b = lbm.Lbm(spec).init(phi0)
        b.set_two_step(True)
        a.step(301)
        b.step(301)
        a.step(299)
        b.step(299)
        assert torch.equal(a.phi(), b.phi())
        wa, _ = a.current()
        wb, _ = b.current()
        assert torch.equal(a.storage_view(a.f[wa]), b.storage_view(b.f[wb]))


def test_two_step_refused_where_it_does_not_apply():
    lbm = _lbm()
    walls = dict(W.spec_nonlinear_2d(70, 30), bc=["periodic", "abb", "periodic"], phi_wall=[[0, 0], [0.3, 0.7], [0, 0]],
                 kpoly=[1.0, 0.0, 0.0, 0.2])   # walls need 3-term polynomials
    d3_cubic = dict(W.d3q19_walls((20, 18, 22))[0], kpoly=[1.0, 0.0, 0.0, 0.5])
    for spec in (d3_cubic, walls):
        s = lbm.Lbm(spec)
        with pytest.raises(lbm.LbmError) as ei:
            s.set_two_step(True)
        assert ei.value.code == lbm.LBM_E_UNSUPPORTED
    assert lbm.Lbm(W.d3q19_walls((20, 18, 22))[0]).two_step_shapes() == [(6, 8), (2, 4)]
    assert lbm.Lbm(W.d3q19_walls((20, 18, 22), precision="f32")[0]).two_step_shapes() == [(14, 16), (6, 8), (2, 4)]
    # tile shapes: 4 for 4- and 2-byte storage, 2 for FP64; the non-default
    # ones need 3-term polynomials
    assert lbm.Lbm(W.spec_nonlinear_2d(100, 37, precision="f32")).two_step_shapes() == \
        [(14, 4), (14, 8), (10, 6), (6, 4)]
    assert lbm.Lbm(W.spec_nonlinear_2d(100, 37, precision="f64")).two_step_shapes() == [(6, 4), (6, 8), (14, 16)]
    for spec, shape in ((W.spec_nonlinear_2d(100, 37, precision="f64"), 3),
                        (W.spec_nonlinear_2d(100, 37, precision="f32"), 4),
                        (W.spec_nonlinear_2d(100, 37, precision="f32", bcoef=0.0) | {"b": [[0, 0, 0, 0.1]] * 2}, 1)):
        s = lbm.Lbm(spec)
        with pytest.raises(lbm.LbmError) as ei:
            s.set_two_step(True, shape)
        assert ei.value.code == lbm.LBM_E_INVALID


# ---------------------------------------------------------------------------
# buffer ownership
# ---------------------------------------------------------------------------

def test_create_allocates_nothing_of_grid_size():
    """lbm_create allocates only the coefficient table and the fixed scratch:
    on a 4096 x 4096 FP32 run with a source (two steps per pass apply, so a
    second history buffer of 64 MiB is needed) the device's free memory drops
    by far less than one N-value buffer, and the second history is reported
    by lbm_state_bytes for the caller to provide."""
    import ctypes
    lbm = _lbm()
    L = lbm.load()
    torch.cuda.synchronize()
    spec = W.spec_nonlinear_2d(4096, 4096, precision="f32")
    d = lbm.desc_from_spec(spec)
    ctx = ctypes.c_void_p()
    free0 = torch.cuda.mem_get_info()[0]
    assert L.lbm_create(ctypes.byref(d), ctypes.byref(ctx)) == 0, L.lbm_last_error()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    fb, pb, p2b = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert L.lbm_state_bytes(ctx, ctypes.byref(fb), ctypes.byref(pb), ctypes.byref(p2b)) == 0
    L.lbm_destroy(ctx)
    n = 4096 * 4096
    say(f"[gpu] lbm_create took {(free0 - free1) / 2**20:.1f} MiB; p {pb.value} p2 {p2b.value}")
    assert free0 - free1 < 16 * 2**20 < 4 * n
    assert pb.value == p2b.value == 4 * n
    # no source: no history is read, so no second buffer is asked for
    d = lbm.desc_from_spec(W.spec_nonlinear_2d(4096, 4096, precision="f32", source=False))
    assert L.lbm_create(ctypes.byref(d), ctypes.byref(ctx)) == 0
    assert L.lbm_state_bytes(ctx, None, None, ctypes.byref(p2b)) == 0
    L.lbm_destroy(ctx)
    assert p2b.value == 0


def test_two_step_without_second_history():
    """A run with a source bound without the second history buffer uses single
    sweeps (same results as with it, bit for bit), and refuses an explicit
    request for two steps per pass with LBM_E_STATE."""
    import ctypes
    lbm = _lbm()
    spec = W.spec_nonlinear_2d(100, 37, precision="f32")
    phi0 = W.noise_field((37, 100), 72)
    say("[gpu] two-step pass without p2")
    a = lbm.Lbm(spec).init(phi0)
    assert a.p2 is not None
    b = lbm.Lbm(spec)
    b.p2 = None
    b.init(phi0)
    with pytest.raises(lbm.LbmError) as ei:
        b.set_two_step(True)
    assert ei.value.code == lbm.LBM_E_STATE
    a.step(37)
    b.step(37)
    assert torch.equal(a.phi(), b.phi())
    # p2 may not alias another buffer
    rc = lbm.load().lbm_init(b.ctx, lbm._ptr(b._phi0), lbm._ptr(b.f[0]), lbm._ptr(b.f[1]), lbm._ptr(b.p),
                             lbm._ptr(b.p), ctypes.c_void_p(0))
    assert rc == lbm.LBM_E_INVALID
