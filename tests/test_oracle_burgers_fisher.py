"""The Burgers-Fisher travelling wave (Sec. 3.2, Eq. 46-51) as a pin of the
oracle's nonlinear Scheme-A path: B(phi) quadratic, R(phi) = b phi (1 - phi)
with the explicit time difference of Remark II, B-tilde = (I - A/2) B' at
each time level, anti-bounce-back walls (Sec. 3.6) whose Dirichlet values
follow the exact solution in time.  The wave runs along the wall axis y and
is uniform across the periodic x axis.

The closed form (the one-dimensional reduction of Eq. 47-48, derived by
substitution like the corrected omega of Eq. 48) is first checked by
substitution into Eq. 46 with finite differences; the oracle's GRE (Eq. 39)
against it must then fall at second order under diffusive refinement
(Fig. 4: slope 2).
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

A_, B_ = 4.0, 1.0
Y0 = -1.0               # the paper's domain [-1, 2] on the wall axis
LENGTH = 3.0


def test_closed_form_satisfies_eq46():
    """Residual of d_t phi + a phi d_y phi - kappa d_yy phi - b phi (1 - phi)
    at the closed form, by central differences of step h (error O(h^2))."""
    for kappa in (0.4, 0.1, 0.03):
        res = []
        for h in (1e-3, 5e-4):
            y = np.linspace(-0.9, 1.9, 57)
            t = 0.37
            f = lambda yy, tt: W.burgers_fisher_wave(yy, tt, A_, B_, kappa)
            ph = f(y, t)
            dt = (f(y, t + h) - f(y, t - h)) / (2 * h)
            dy = (f(y + h, t) - f(y - h, t)) / (2 * h)
            dyy = (f(y + h, t) - 2 * ph + f(y - h, t)) / (h * h)
            r = dt + A_ * ph * dy - kappa * dyy - B_ * ph * (1 - ph)
            res.append(np.abs(r).max())
        # second-order decay of the difference error: the exact residual is 0
        assert res[1] < 0.3 * res[0] + 1e-9, (kappa, res)
        assert res[1] < 1e-4 * max(1.0, A_ / kappa), (kappa, res)
    # and a form with the 2-D omega of Eq. 48 as printed (one factor (delta+1)
    # short) does not satisfy the 1-D equation: the substitution is sensitive
    kappa, h, y, t = 0.4, 1e-4, np.linspace(-0.9, 1.9, 57), 0.37
    Aw = -A_ / (4 * kappa)
    om_bad = (A_ * A_ + 2 * B_ * kappa) / (2 * A_)
    g = lambda yy, tt: 0.5 + 0.5 * np.tanh(Aw * (yy - om_bad * tt))
    ph = g(y, t)
    r = ((g(y, t + h) - g(y, t - h)) / (2 * h) + A_ * ph * (g(y + h, t) - g(y - h, t)) / (2 * h)
         - kappa * (g(y + h, t) - 2 * ph + g(y - h, t)) / (h * h) - B_ * ph * (1 - ph))
    assert np.abs(r).max() > 1e-2


def run_wave(n, kappa, T, nx=2, scheme="A", snap=None):
    """Oracle run of the wave on n nodes along y; returns (phi(T), exact, dt)."""
    spec, dx, dt = W.spec_burgers_fisher(n, nx=nx, a=A_, b=B_, kappa=kappa, length=LENGTH, scheme=scheme)
    p = orc.params_from_spec(spec)
    y = Y0 + (np.arange(n) + 0.5) * dx
    exact = lambda tt: W.burgers_fisher_wave(y, tt, A_, B_, kappa)
    wall = lambda tt: (float(W.burgers_fisher_wave(Y0, tt, A_, B_, kappa)),
                       float(W.burgers_fisher_wave(Y0 + LENGTH, tt, A_, B_, kappa)))
    nst = int(round(T / dt))
    phi0 = np.repeat(exact(0.0)[:, None], nx, axis=1)
    f, pp = orc.init(p, phi0)
    for t in range(nst):
        # push-form streaming of step t (t -> t + 1): wall values at t + 1/2
        p.phi_wall[1][0], p.phi_wall[1][1] = wall((t + 0.5) * dt)
        orc.step(p, f, pp)
    ph = orc.phi(p, f)
    return ph, np.repeat(exact(nst * dt)[:, None], nx, axis=1), dt


def gre(num, ana):
    return float(np.abs(ana - num).sum() / np.abs(ana).sum())


@pytest.mark.parametrize("kappa,ns", [(0.4, (48, 96, 192)), (0.1, (96, 192, 384))])
def test_burgers_fisher_second_order(kappa, ns):
    """GRE at T = 0.5 (the front crosses the middle of the domain) for three
    resolutions; Pe = L a / kappa = 30 and 120.  Fitted orders 2 +- 0.3."""
    gres = []
    for n in ns:
        ph, ex, _ = run_wave(n, kappa, 0.5)
        assert np.abs(ph - ph[:, :1]).max() < 1e-13          # uniform across x
        gres.append(gre(ph, ex))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(len(gres) - 1)]
    print(f"Burgers-Fisher kappa={kappa}: GRE {gres}, orders {order}")
    assert gres[-1] < 2e-3
    assert all(1.7 <= o <= 2.3 for o in order), (gres, order)


def test_burgers_fisher_scheme_b_second_order():
    """The paper's default scheme on the same wave: Scheme B, whose Eq. 35 is
    implicit for R = b phi (1 - phi) (solved by the oracle's Newton step).
    Second order, and close to the Scheme-A errors."""
    gres = []
    for n in (48, 96, 192):
        ph, ex, _ = run_wave(n, 0.4, 0.5, scheme="B")
        gres.append(gre(ph, ex))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(2)]
    print(f"Burgers-Fisher Scheme B: GRE {gres}, orders {order}")
    assert gres[-1] < 2e-3
    assert all(1.7 <= o <= 2.3 for o in order), (gres, order)
