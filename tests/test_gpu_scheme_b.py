"""Scheme B (Eq. 33-35) and per-node fields on the GPU, against the oracle.

Scheme B stores fbar = f - R_k / 2, evolves it by Eq. 34 with Btilde = B'
and recovers phi by Eq. 35; R may be a polynomial of degree <= 2 in phi
(Eq. 35 then implicit, solved in closed form on the GPU and by Newton's
method in the oracle) plus an external field R(x, t).  A per-node K0(x) field gives A per node by Eq. 26
(Sec. 3.5).  Cases: equal-rate and moment-space collisions, walls, D3Q19, the
time-dependent source of Sec. 3.1 (rewritten on the device between steps),
the variable diffusion tensor of Sec. 3.5, and reduced-precision storage.
    FP64 <= 1e-12 against the oracle, FP32 <= 1e-5 (relative L2 and
    max |d| / max |phi|).
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


def rel(a, b):
    a = np.asarray(a.cpu() if hasattr(a, "cpu") else a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def k_compact(kf, dim):
    """[..., 3, 3] full tensors -> the ABI's per-node (xx, yy, xy) / (xx, yy, zz, xy, yz, xz)."""
    if dim == 2:
        return np.stack([kf[..., 0, 0], kf[..., 1, 1], kf[..., 0, 1]], axis=-1)
    return np.stack([kf[..., 0, 0], kf[..., 1, 1], kf[..., 2, 2], kf[..., 0, 1], kf[..., 1, 2], kf[..., 0, 2]],
                    axis=-1)


def gpu_run(spec, phi0, snapshots, kfield=None, source=None, flags=0):
    """GPU run with optional K0 field ([..., 3, 3]) and source(t) -> R(x, t);
    the source tensor is rewritten on the device before every step."""
    from paper_1603_09577_amd import lbm
    sim = lbm.Lbm(spec, flags=flags)
    dim = 2 if spec["lattice"] == 9 else 3
    kt = None if kfield is None else torch.tensor(k_compact(np.asarray(kfield), dim), dtype=torch.float64,
                                                   device="cuda").contiguous()
    rt = None if source is None else torch.tensor(source(0), dtype=torch.float64, device="cuda").contiguous()
    sim.set_fields(kt, rt)
    sim.init(phi0)
    out = {}
    t = 0
    for s in sorted(snapshots):
        if source is None:
            sim.step(s - t)
            t = s
        else:
            while t < s:
                sim.step(1)
                t += 1
                rt.copy_(torch.as_tensor(source(t), dtype=torch.float64))
        out[s] = sim.phi().cpu().numpy()
    return out


def oracle_snaps(spec, phi0, snapshots, kfield=None, source=None):
    p = orc.params_from_spec(dict(spec, precision="f64"))
    _, snaps = orc.run(p, phi0, max(snapshots), snapshots=tuple(snapshots), source=source, kfield=kfield)
    return snaps


def compare(name, spec, phi0, snapshots, tol, **kw):
    flags = kw.pop("flags", 0)
    say(f"[gpu scheme B] {name} shape={spec['shape']} prec={spec.get('precision', 'f64')} steps={snapshots}")
    got = gpu_run(spec, phi0, snapshots, flags=flags, **kw)
    ref = oracle_snaps(spec, phi0, snapshots, **kw)
    errs = {s: rel(got[s], ref[s]) for s in snapshots}
    pts = {s: float(np.abs(got[s] - ref[s]).max() / np.abs(ref[s]).max()) for s in snapshots}
    say("    rel L2 " + "  ".join(f"{s}: {e:.2e}" for s, e in errs.items()))
    say("    max |d| / max |phi| " + "  ".join(f"{s}: {e:.2e}" for s, e in pts.items()))
    assert max(errs.values()) <= tol, errs
    assert max(pts.values()) <= tol, pts


def _nonlinear_b(nx, ny, precision="f64"):
    spec = W.spec_nonlinear_2d(nx, ny, source=False, precision=precision)
    spec["scheme"] = "B"
    spec["rpoly"] = [2e-4]
    return spec


@pytest.mark.parametrize("flags", [0, 1])
def test_scheme_b_constant_source_nonlinear(flags):
    """Nonlinear B and K(phi), constant R: equal-rate (flags 0) and moment-space
    (flags 1) forms, ragged grid."""
    spec = _nonlinear_b(37, 29)
    compare(f"nonlinear constant R flags={flags}", spec, W.noise_field((29, 37), 31), (1, 7, 60, 250), 1e-12,
            flags=flags)


def test_scheme_b_general_rates_walls():
    spec = _nonlinear_b(23, 31)
    spec["bc"] = ["periodic", "abb", "periodic"]
    spec["phi_wall"] = [[0, 0], [0.3, 0.65], [0, 0]]
    spec["s"] = [0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05]
    compare("general rates, walls", spec, W.noise_field((31, 23), 32), (1, 9, 120), 1e-12)


def test_scheme_b_d3q19_walls_source_field_kfield():
    n = (14, 11, 17)
    spec = W.spec_d3q19_aniso(n, phi_wall=0.2)
    spec["scheme"] = "B"
    spec["rpoly"] = [1e-4]
    phi0 = W.gaussians_3d(n, 7)
    rng = np.random.default_rng(33)
    kf = np.zeros(n[::-1] + (3, 3))
    for z in range(n[2]):
        kf[z] = W.random_spd3(100 + z)
    rfield = 1e-4 * rng.uniform(-1, 1, n[::-1])
    compare("d3q19 walls, K0 field, source field", spec, phi0, (1, 5, 40), 1e-12, kfield=kf,
            source=lambda t: rfield)


# ---------------------------------------------------------------------------
# Scheme B with R depending on phi (Eq. 35 solved at every node)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("flags,prec,tol", [(0, "f64", 1e-12), (1, "f64", 1e-12), (0, "f32", 1e-5),
                                            (1, "f32", 1e-5)])
def test_scheme_b_implicit_source_nonlinear(flags, prec, tol):
    """The nonlinear 2-D workload's physics (B = 0.5 phi^2 (1, 1), K = K0 (1 +
    phi^2), R = 0.1 phi (1 - phi) in its grid units) in Scheme B: the closed-
    form root of Eq. 35 on the GPU against the oracle's Newton solve;
    equal-rate (flags 0) and moment-space (flags 1) collisions."""
    spec = W.spec_nonlinear_2d(37, 29, precision=prec)
    spec["scheme"] = "B"
    compare(f"implicit R(phi) flags={flags}", spec, W.noise_field((29, 37), 34), (1, 7, 60, 300), tol,
            flags=flags)


def test_scheme_b_implicit_walls_field_d2q9():
    """R(phi) plus an external field, walls with unequal rates."""
    spec = W.spec_nonlinear_2d(23, 31)
    spec.update(scheme="B", bc=["periodic", "abb", "periodic"], phi_wall=[[0, 0], [0.3, 0.65], [0, 0]],
                s=[0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05], rpoly=[1e-4, 2e-3, -3e-3])
    rng = np.random.default_rng(35)
    rfield = 1e-4 * rng.uniform(-1, 1, (31, 23))
    compare("implicit R(phi) + field, walls", spec, W.noise_field((31, 23), 36), (1, 9, 120), 1e-12,
            source=lambda t: rfield)


def test_scheme_b_implicit_d3q19():
    n = (13, 11, 15)
    spec = W.spec_d3q19_aniso(n, phi_wall=0.2)
    spec.update(scheme="B", rpoly=[0.0, 0.01, -0.01], phi_ref=0.3)
    spec["s"] = [0.0] + [1.0 + 0.04 * i for i in range(18)]
    compare("d3q19 implicit R(phi), unequal rates", spec, W.gaussians_3d(n, 8), (1, 5, 40), 1e-12)
    spec32 = dict(spec, precision="f32", s=[0.0] + [1.0] * 18)
    compare("d3q19 implicit R(phi) f32", spec32, W.gaussians_3d(n, 8), (1, 40), 1e-5)


def test_scheme_b_implicit_full_size():
    """The 1024 x 1024 nonlinear workload in Scheme B, a few steps at full size."""
    spec, phi0, _ = W.nonlinear_2d(1024)
    spec["scheme"] = "B"
    compare("nonlinear2d-1024 scheme B", spec, phi0, (1, 4), 1e-12)
    spec32 = dict(spec, precision="f32")
    compare("nonlinear2d-1024 scheme B f32", spec32, phi0, (4,), 1e-5)


def _channel_spec(N, s1, s3, ux, precision="f64"):
    kap = (1 / s3 - 0.5) / 3
    s = [s1] * 9
    s[0] = 0.0
    return dict(lattice=9, shape=(3, N), bc=["periodic", "abb", "periodic"],
                phi_wall=[[0, 0], [0.0, 1.0], [0, 0]], scheme="B", d=1.0, s=s,
                b=[[0, ux], [0, 0]], dpoly=[0, 1], dten=np.eye(3).tolist(),
                k0=(kap * np.eye(3)).tolist(), kpoly=[1.0], rpoly=[2 * kap / N ** 2],
                precision=precision, phi_ref=0.5), kap


@pytest.mark.parametrize("N,s1,s3,ux", [(4, 1.0, 0.6, 0.1), (8, 1.3, 0.9, 0.1), (8, 0.7, 1.9, 0.0)])
def test_channel_exact_discrete_solution(N, s1, s3, ux):
    """Sec. 3.6 (X6): Scheme B with R = 2 kappa dphi / L^2 between anti-bounce-
    back walls at phi = 0 and 1.  The steady state on the GPU equals the exact
    discrete solution (Eq. 71 with the sign of Eq. 70, phi_s of Eq. 72b)."""
    from paper_1603_09577_amd import lbm
    spec, kap = _channel_spec(N, s1, s3, ux)
    sim = lbm.Lbm(spec).init(np.full((N, 3), 0.5))
    sim.step(int(30 * N * N / kap) + 1024)
    ph = sim.phi().cpu().numpy()[:, 0]
    yb = (np.arange(1, N + 1) - 0.5) / N
    phis = 1.0 / (12 * N ** 2 * s1 * s3) * (s1 * s3 - 8 * (s1 + s3) + 16)
    err = np.abs(ph - (yb * (2 - yb) + phis)).max()
    say(f"[gpu scheme B] channel N={N} s1={s1} s3={s3} ux={ux}: max |phi - exact| = {err:.2e}")
    assert err < 1e-12


def test_sine_wave_time_dependent_source():
    """Sec. 3.1 (Eq. 42-45): the source of Eq. 43 rewritten on the device before
    every step; against the oracle, and second order in space on the GPU."""
    kap, ux, uy, L = 0.002, 0.1, 0.1, 2.0
    klat = 1.0 / 24.0
    g = 1 - 2 * math.pi ** 2 * kap

    def setup(n):
        dx = L / n
        dt = klat * dx * dx / kap
        spec = dict(lattice=9, shape=(n, n), bc=["periodic"] * 3, scheme="B", d=1.0,
                    s=[0.0] + [1.0] * 8, b=[[0.0, ux * dt / dx], [0.0, uy * dt / dx]],
                    dpoly=[0, 1], dten=np.eye(3).tolist(), k0=(klat * np.eye(3)).tolist(),
                    kpoly=[1.0], rpoly=[])
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")
        body = np.sin(math.pi * (X + Y)) + math.pi * (ux + uy) * np.cos(math.pi * (X + Y))
        return spec, dt, np.sin(math.pi * (X + Y)), (lambda s: dt * math.exp(g * s * dt) * body)

    spec, dt, phi0, src = setup(40)
    compare("sine wave, R(x, t)", spec, phi0, (1, 13, 80), 1e-12, source=src)
    gres = []
    for r in (1, 2, 4):
        n = 32 * r
        spec, dt, phi0, src = setup(n)
        nst = 10 * r * r
        got = gpu_run(spec, phi0, (nst,), source=src)[nst]
        exact = math.exp(g * nst * dt) * phi0
        gres.append(float(np.abs(got - exact).sum() / np.abs(exact).sum()))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(2)]
    say(f"    GRE {gres}, order {order}")
    assert all(1.7 < o < 2.3 for o in order)


def test_variable_diffusion_tensor_field():
    """Sec. 3.5 (Eq. 64-68): K(x) = kappa diag(2 - sin 2pi x sin 2pi y, 1) as a
    per-node field with the source of Eq. 66; against the oracle (FP64 and
    FP32) and second order in space on the GPU."""
    kap, u = 1e-3, 0.1
    klat = 1.0 / 24.0
    g = 1 - 12 * np.pi ** 2 * kap

    def setup(n, precision="f64"):
        dx = 1.0 / n
        dt = klat * dx * dx / kap
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")
        sxy = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        kf = np.zeros((n, n, 3, 3))
        kf[..., 0, 0] = klat * (2 - sxy)
        kf[..., 1, 1] = klat
        kf[..., 2, 2] = klat
        spec = dict(lattice=9, shape=(n, n), bc=["periodic"] * 3, scheme="B", d=1.0,
                    s=[0.0] + [1.0] * 8, b=[[0.0, u * dt / dx], [0.0, u * dt / dx]],
                    dpoly=[0, 1], dten=np.eye(3).tolist(), k0=(klat * np.eye(3)).tolist(),
                    kpoly=[1.0], rpoly=[], precision=precision)
        body = (sxy + 4 * kap * np.pi ** 2 * np.cos(4 * np.pi * X) * np.sin(2 * np.pi * Y) ** 2
                + 2 * np.pi * (u * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
                               + u * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)))
        return spec, dt, sxy, kf, (lambda s: dt * math.exp(g * s * dt) * body)

    spec, dt, phi0, kf, src = setup(48)
    compare("variable K(x) field", spec, phi0, (1, 9, 70), 1e-12, kfield=kf, source=src)
    spec32, dt, phi0, kf, src = setup(48, "f32")
    compare("variable K(x) field fp32", spec32, phi0, (1, 9, 70), 1e-5, kfield=kf, source=src)
    gres = []
    for r in (1, 2, 4):
        n = 24 * r
        spec, dt, phi0, kf, src = setup(n)
        nst = 12 * r * r
        got = gpu_run(spec, phi0, (nst,), kfield=kf, source=src)[nst]
        exact = math.exp(g * nst * dt) * phi0
        gres.append(float(np.abs(got - exact).sum() / np.abs(exact).sum()))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(2)]
    say(f"    GRE {gres}, order {order}")
    assert all(1.7 < o < 2.3 for o in order)


def test_scheme_a_with_k_field():
    """A K0 field under Scheme A with the nonlinear source: per-node A at both
    time levels of the source."""
    spec = W.spec_nonlinear_2d(33, 26)
    rng = np.random.default_rng(34)
    kf = np.zeros((26, 33, 3, 3))
    k0 = np.asarray(spec["k0"])
    scale = 1 + 0.5 * rng.uniform(-1, 1, (26, 33))
    kf[..., :2, :2] = k0[:2, :2] * scale[..., None, None]
    kf[..., 2, 2] = 1.0
    compare("scheme A, K0 field", spec, W.noise_field((26, 33), 35), (1, 11, 90), 1e-12, kfield=kf)


@pytest.mark.parametrize("precision,tol", [("f32", 1e-5), ("f16", 2e-2)])
def test_scheme_b_reduced_storage(precision, tol):
    spec = _nonlinear_b(41, 30, precision=precision)
    compare(f"scheme B {precision}", spec, W.noise_field((30, 41), 36), (1, 50, 300), tol)


def test_refusals():
    from paper_1603_09577_amd import lbm
    # an external source field needs Scheme B
    spec = W.spec_nonlinear_2d(16, 12)
    sim = lbm.Lbm(spec)
    rf = torch.zeros(12 * 16, dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LbmError) as ei:
        sim.set_fields(None, rf)
    assert ei.value.code == lbm.LBM_E_UNSUPPORTED
    # no adjoint with a K0 field
    kf = torch.zeros(12 * 16 * 3, dtype=torch.float64, device="cuda")
    kf[0::3] = 0.02
    kf[1::3] = 0.01
    sim.set_fields(kf, None)
    sim.init(W.noise_field((12, 16), 37))
    psi, pi = sim.adjoint_buffers()
    with pytest.raises(lbm.LbmError) as ei:
        sim.adjoint_seed(torch.ones(sim.shape, dtype=torch.float64, device="cuda"), psi, pi)
    assert ei.value.code == lbm.LBM_E_UNSUPPORTED
    # Scheme B solves Eq. 35 in closed form for R of degree <= 2 only
    spec_b = _nonlinear_b(16, 12)
    spec_b["rpoly"] = [0.0, 1e-3, 0.0, -1e-3]
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lbm(spec_b)
    assert ei.value.code == lbm.LBM_E_UNSUPPORTED
    # and the adjoint refuses Scheme B sources, also R(phi)
    spec_b["rpoly"] = [0.0, 1e-3, -1e-3]
    sim = lbm.Lbm(spec_b).init(W.noise_field((12, 16), 38))
    psi, pi = sim.adjoint_buffers()
    with pytest.raises(lbm.LbmError) as ei:
        sim.adjoint_seed(torch.ones(sim.shape, dtype=torch.float64, device="cuda"), psi, pi)
    assert ei.value.code == lbm.LBM_E_UNSUPPORTED
