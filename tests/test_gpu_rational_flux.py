"""Remark III with a rational flux on the GPU (lbm_desc.bden): the
Buckley-Leverett flux of Sec. 3.3 (Eq. 54), B = (f, g) with f and g sharing
the denominator phi^2 + (1 - phi)^2.

  * parity with the oracle: Scheme A with R(phi) and Scheme B with an external
    field, equal-rate and moment-space collisions, walls, D3Q19 with a
    three-component rational B; FP64 <= 1e-12, FP32 <= 1e-5 (relative L2 and
    max |d| / max |phi|);
  * the manufactured solution of tests/test_oracle_rational_flux.py on the GPU:
    second order, 2 +- 0.3;
  * Sec. 3.3 at the paper's size (301 x 301 on [-1.5, 1.5]^2, kappa = 0.1 and
    0.01, T = 0.5; the problem has no closed form): sum phi conserved on the
    periodic grid and phi stays within [0, 1] up to a few per cent;
  * a rational B without LBM_FLAG_REMARK3 is refused.
"""
import math
import sys

import numpy as np
import pytest

import oracle as orc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BL_NUM = [[0.0, 0.0, 1.0], [0.0, 0.0, -4.0, 10.0, -5.0]]
BL_DEN = [1.0, -2.0, 2.0]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def spec_bl(nx, ny, scale, kl, scheme="A", rpoly=(), precision="f64", phi_ref=0.5):
    return dict(lattice=9, shape=(nx, ny), bc=["periodic"] * 3, scheme=scheme, d=1.0, s=[0.0] + [1.0] * 8,
                b=[[scale * v for v in BL_NUM[0]], [scale * v for v in BL_NUM[1]]], bden=BL_DEN,
                dpoly=[0.0, 1.0], dten=np.eye(3).tolist(), k0=(kl * np.eye(3)).tolist(), kpoly=[1.0],
                rpoly=list(rpoly), variant="remark3", precision=precision, phi_ref=phi_ref)


def run_both(spec, phi0, steps, flags=0, source=None):
    from paper_1603_09577_amd import lbm
    sim = lbm.Lbm(spec, flags=flags)
    rt = None
    if source is not None:
        rt = torch.tensor(source(0), dtype=torch.float64, device="cuda").contiguous()
        sim.set_fields(None, rt)
    sim.init(phi0)
    for t in range(steps):
        sim.step(1)
        if source is not None:
            rt.copy_(torch.as_tensor(source(t + 1), dtype=torch.float64))
    got = sim.phi().cpu().numpy()
    ref, _ = orc.run(orc.params_from_spec(dict(spec, precision="f64")), phi0, steps, source=source)
    return got, ref


def check(name, got, ref, tol):
    e2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    ep = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"[gpu rational B] {name}: rel L2 {e2:.2e}, max |d| / max |phi| {ep:.2e}")
    assert np.isfinite(got).all()
    assert e2 <= tol and ep <= tol


@pytest.mark.parametrize("flags,prec,tol", [(0, "f64", 1e-12), (1, "f64", 1e-12), (0, "f32", 1e-5)])
def test_buckley_leverett_scheme_a_against_oracle(flags, prec, tol):
    rng = np.random.default_rng(81)
    phi0 = 0.5 + 0.3 * rng.uniform(-1, 1, (29, 37))
    spec = spec_bl(37, 29, 0.1, 0.08, rpoly=[0.0, 0.002, -0.002], precision=prec)
    got, ref = run_both(spec, phi0, 120, flags)
    check(f"Scheme A flags={flags} {prec}", got, ref, tol)


def test_buckley_leverett_scheme_b_walls_field():
    rng = np.random.default_rng(82)
    phi0 = 0.5 + 0.3 * rng.uniform(-1, 1, (31, 23))
    spec = spec_bl(23, 31, 0.1, 0.08, scheme="B", rpoly=[1e-4])
    spec.update(bc=["periodic", "abb", "periodic"], phi_wall=[[0, 0], [0.2, 0.9], [0, 0]],
                s=[0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05])
    field = 1e-4 * rng.uniform(-1, 1, (31, 23))
    got, ref = run_both(spec, phi0, 90, source=lambda t: field)
    check("Scheme B, walls, unequal rates, source field", got, ref, 1e-12)


def test_rational_flux_d3q19():
    n = (11, 9, 13)
    rng = np.random.default_rng(83)
    phi0 = 0.5 + 0.2 * rng.uniform(-1, 1, n[::-1])
    spec = dict(lattice=19, shape=n, bc=["periodic", "periodic", "abb"], phi_wall=[[0, 0], [0, 0], [0.3, 0.6]],
                scheme="A", d=1.0, s=[0.0] + [1.0 + 0.03 * i for i in range(18)],
                b=[[0.0, 0.0, 0.05], [0.0, 0.02, 0.0, 0.03], [0.0, -0.03, 0.02]], bden=[1.0, -0.5, 0.5],
                dpoly=[0.0, 1.0], dten=np.eye(3).tolist(), k0=(0.03 * np.eye(3)).tolist(), kpoly=[1.0, 0.2],
                rpoly=[0.0, 0.003, -0.003], variant="remark3", phi_ref=0.5)
    got, ref = run_both(spec, phi0, 40)
    check("D3Q19, walls, unequal rates", got, ref, 1e-12)


def _cstep(fn, p):
    return np.imag(fn(p + 1j * 1e-30)) / 1e-30


def bl_f(p):
    return p * p / (p * p + (1 - p) ** 2)


def bl_g(p):
    return bl_f(p) * (1 - 5 * (1 - p) ** 2)


def test_manufactured_solution_second_order_on_gpu():
    from paper_1603_09577_amd import lbm
    kappa, T = 0.05, 0.2
    gres = []
    for n in (32, 64, 128):
        dx = 1.0 / n
        dt = 0.16 * dx * dx / kappa
        spec = spec_bl(n, n, dt / dx, kappa * dt / dx ** 2, scheme="B")
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")
        s2, c2 = np.sin(2 * math.pi * Y), np.cos(2 * math.pi * Y)

        def source(step):
            t = step * dt
            s1, c1 = np.sin(2 * math.pi * (X - t)), np.cos(2 * math.pi * (X - t))
            ph = 0.5 + 0.25 * s1 * s2
            R = (-0.5 * math.pi * c1 * s2 + _cstep(bl_f, ph) * 0.5 * math.pi * c1 * s2
                 + _cstep(bl_g, ph) * 0.5 * math.pi * s1 * c2 + kappa * 2 * (2 * math.pi) ** 2 * 0.25 * s1 * s2)
            return dt * R

        nst = int(round(T / dt))
        sim = lbm.Lbm(spec)
        rt = torch.tensor(source(0), device="cuda").contiguous()
        sim.set_fields(None, rt)
        sim.init(0.5 + 0.25 * np.sin(2 * math.pi * X) * s2)
        for t in range(nst):
            sim.step(1)
            rt.copy_(torch.as_tensor(source(t + 1)))
        ex = 0.5 + 0.25 * np.sin(2 * math.pi * (X - nst * dt)) * s2
        got = sim.phi().cpu().numpy()
        gres.append(float(np.abs(got - ex).sum() / np.abs(ex).sum()))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(2)]
    say(f"[gpu rational B] manufactured solution: GRE {gres}, orders {order}")
    assert all(1.7 <= o <= 2.3 for o in order), (gres, order)


@pytest.mark.parametrize("kappa", [0.1, 0.01])
def test_buckley_leverett_paper_size(kappa):
    """Sec. 3.3: [-1.5, 1.5]^2, 301 x 301 (300 distinct periodic nodes), phi0 =
    1 inside x^2 + y^2 < 0.5, T = 0.5.  Lattice speed c = 10 (|B'| of Eq. 54
    reaches about 2.3, beyond what c = 1 allows)."""
    from paper_1603_09577_amd import lbm
    n, L, c = 300, 3.0, 10.0
    dx = L / n
    dt = dx / c
    x = -1.5 + (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    phi0 = np.where(X * X + Y * Y < 0.5, 1.0, 0.0)
    spec = spec_bl(n, n, dt / dx, kappa * dt / dx ** 2)
    sim = lbm.Lbm(spec).init(phi0)
    nst = int(round(0.5 / dt))
    sim.step(nst)
    ph = sim.phi().cpu().numpy()
    mass = abs(ph.sum() - phi0.sum()) / phi0.sum()
    say(f"[paper] Sec. 3.3 Buckley-Leverett kappa = {kappa}: {nst} steps, mass drift {mass:.2e}, "
        f"phi in [{ph.min():.4f}, {ph.max():.4f}], centre line {ph[n // 2, n // 2]:.4f}")
    assert np.isfinite(ph).all()
    assert mass < 1e-12
    assert -0.05 < ph.min() and ph.max() < 1.05


def test_rational_flux_refused_without_remark3():
    from paper_1603_09577_amd import lbm
    spec = spec_bl(16, 12, 0.1, 0.1)
    spec["variant"] = "standard"
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Lbm(spec)
    assert ei.value.code == lbm.LBM_E_UNSUPPORTED
