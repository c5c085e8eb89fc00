"""The paper's own experiments on the GPU path, at the paper's sizes, against
the errors it prints (tests/golden/paper_values.json).

Readings (the paper leaves them open): lattice speed c = 1 (delta t = delta
x), and a "401 x 401" periodic lattice has 400 distinct nodes per axis (node
400 is node 0).  Rates not tied to K are 1.0 (Eq. 41) unless stated, d = 1,
Scheme B (the paper's default; without a source it equals Scheme A).  GRE is
Eq. 39.  Each run is FP64; its per-step parity with the oracle is covered
elsewhere, so these numbers are the oracle's too.

    Sec. 3.4, Gaussian hill, isotropic K: matches the printed 1.199e-4 to all
      four digits in both approaches; anisotropic K within 3 %.
    Sec. 3.6, stability at kappa = 1e-4: MRT (s = 0.6) gives the printed
      4.438e-2 to four digits; BGK diverges.
    Sec. 3.5, variable K(x): within 10 % at Pe = 100; Pe = 1000 is reported
      only (the stated kappa = 1e-3 cannot give Pe = 1000 at u = 0.1).
"""
import json
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PAPER = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gre(num, ana):
    return float(np.abs(ana - num).sum() / np.abs(ana).sum())


def hill_exact(X, Y, K, u, T, s0, L=2.0):
    """Eq. 60 (with the nearest periodic images; they are below 1e-40 here)."""
    sig = s0 * s0 * np.eye(2) + 2 * np.asarray(K) * T
    si = np.linalg.inv(sig)
    out = np.zeros_like(X)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            dx = X - u[0] * T - i * L
            dy = Y - u[1] * T - j * L
            out += np.exp(-(si[0, 0] * dx * dx + 2 * si[0, 1] * dx * dy + si[1, 1] * dy * dy) / 2)
    return out * s0 * s0 / math.sqrt(abs(np.linalg.det(sig)))


def hill_run(K, approach, u=(0.01, 0.01), T=10.0, s_other=1.0, kappa=1e-3, bgk=False, n=400):
    """Sec. 3.4 on [-1, 1]^2: sigma0 = 0.01, phi0 = 2 pi sigma0^2 (unit peak)."""
    from paper_1603_09577_amd import lbm
    L = 2.0
    dx = L / n
    dt = dx
    x = -1 + np.arange(n) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    s0 = 0.01
    K = np.asarray(K, float)
    dten = np.eye(3)
    if approach == 1:
        kl = K * dt / dx ** 2
    else:                     # Eq. 62: K = kappa I in S, D = K phi / kappa
        kl = kappa * np.eye(2) * dt / dx ** 2
        dten[:2, :2] = K / kappa
    k3 = np.eye(3) * kl[0, 0]
    k3[:2, :2] = kl
    s = [0.0] + [s_other] * 8
    if bgk:                   # one rate for every moment: the BGK model
        s = [0.0] + [1.0 / (3 * kl[0, 0] + 0.5)] * 8
    spec = dict(lattice=9, shape=(n, n), bc=["periodic"] * 3, scheme="B", d=1.0, s=s,
                b=[[0.0, u[0] * dt / dx], [0.0, u[1] * dt / dx]], dpoly=[0, 1], dten=dten.tolist(),
                k0=k3.tolist(), kpoly=[1.0], rpoly=[])
    sim = lbm.Lbm(spec).init(np.exp(-(X * X + Y * Y) / (2 * s0 * s0)))
    nst = int(round(T / dt))
    sim.step(nst)
    ph = sim.phi().cpu().numpy()
    if not np.isfinite(ph).all():
        return float("inf")
    return gre(ph, hill_exact(X, Y, K, u, nst * dt, s0))


@pytest.mark.parametrize("approach", [1, 2])
def test_gaussian_hill_printed_errors(approach):
    printed = PAPER[f"gaussian_hill_gre_approach{approach}"]["value"]
    tensors = (np.eye(2), np.diag([1.0, 2.0]), np.array([[1.0, 1.0], [1.0, 2.0]]))
    for name, K, pv in zip(("isotropic", "diagonal", "full"), tensors, printed):
        g = hill_run(K * 1e-3, approach)
        say(f"[paper] Sec. 3.4 approach {approach} {name}: GRE {g:.4e}, printed {pv:.4e} ({g / pv - 1:+.2%})")
        tol = 2e-3 if name == "isotropic" else 3e-2
        assert abs(g / pv - 1) <= tol


def test_stability_mrt_versus_bgk():
    ref = PAPER["stability_kappa_1e-4"]["value"]
    K = np.array([[1.0, 1.0], [1.0, 2.0]])
    for kap in (1e-3, 1e-4):
        g = hill_run(K * kap, 2, u=(0.1, 0.1), T=5.0, s_other=0.6, kappa=kap)
        gb = hill_run(K * kap, 2, u=(0.1, 0.1), T=5.0, kappa=kap, bgk=True)
        say(f"[paper] Sec. 3.6 kappa {kap:g}: MRT GRE {g:.4e}, BGK GRE {gb:.4e}")
        if kap == 1e-4:
            assert abs(g / ref["mrt_gre"] - 1) <= 2e-3
            assert not gb < 1.0          # BGK blows up (non-finite or huge)
        else:
            assert g < 0.05 and gb < 0.05   # both stable at kappa = 1e-3


def test_variable_diffusion_tensor_printed_errors():
    from paper_1603_09577_amd import lbm
    printed = PAPER["variable_k_gre"]["value"]
    for kap, key in ((1e-3, "pe_100"), (1e-4, "pe_1000")):
        n, u = 400, 0.1
        dx = 1.0 / n
        dt = dx
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")
        sxy = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        kl = kap * dt / dx ** 2
        kf = np.stack([kl * (2 - sxy), np.full_like(sxy, kl), np.zeros_like(sxy)], axis=-1)
        spec = dict(lattice=9, shape=(n, n), bc=["periodic"] * 3, scheme="B", d=1.0, s=[0.0] + [1.0] * 8,
                    b=[[0.0, u * dt / dx], [0.0, u * dt / dx]], dpoly=[0, 1], dten=np.eye(3).tolist(),
                    k0=(kl * np.eye(3)).tolist(), kpoly=[1.0], rpoly=[])
        g = 1 - 12 * np.pi ** 2 * kap
        body = torch.tensor(sxy + 4 * kap * np.pi ** 2 * np.cos(4 * np.pi * X) * np.sin(2 * np.pi * Y) ** 2
                            + 2 * np.pi * (u * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
                                           + u * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)), device="cuda")
        rf = (dt * body).contiguous()
        sim = lbm.Lbm(spec)
        sim.set_fields(torch.tensor(kf, device="cuda").contiguous(), rf)
        sim.init(sxy)
        nst = int(round(3.0 / dt))
        for t in range(nst):          # Eq. 66 at the next time level, rewritten on the device
            sim.step(1)
            rf.copy_(dt * math.exp(g * (t + 1) * dt) * body)
        e = gre(sim.phi().cpu().numpy(), math.exp(g * nst * dt) * sxy)
        pv = printed[key]
        say(f"[paper] Sec. 3.5 kappa {kap:g}: GRE {e:.4e}, printed {pv:.4e} ({e / pv - 1:+.1%})")
        if key == "pe_100":
            assert abs(e / pv - 1) <= 0.1
        else:
            assert e < 1e-3
