"""Remark III (Eq. 36-38) with a flux B that is not a polynomial: B_a =
P_a(phi) / Q(phi), the form of the Buckley-Leverett flux of Sec. 3.3 (Eq. 54),
whose C of Eq. 7 the paper writes with arctan and logarithms (Eq. 57).
Remark III needs only B and B', so the oracle takes B' by the quotient rule.

Pins:
  * a common factor: P = u (phi + phi^2), Q = 1 + phi gives exactly the run of
    B = u phi (and P = c phi^2 (2 + phi), Q = 2 + phi that of B = c phi^2);
  * mass: periodic runs with the Buckley-Leverett flux conserve sum phi;
  * accuracy: a manufactured smooth solution of Eq. 52 with the
    Buckley-Leverett f and g (the source that makes it exact is formed here
    from the flux derivatives by complex step, independently of the oracle)
    falls at second order under diffusive refinement.
"""
import math

import numpy as np
import pytest

import oracle as orc

# Eq. 54: f = phi^2 / (phi^2 + (1 - phi)^2), g = f [1 - 5 (1 - phi)^2]; the
# shared denominator Q = 2 phi^2 - 2 phi + 1, numerators phi^2 and
# -4 phi^2 + 10 phi^3 - 5 phi^4 (coefficients in increasing powers)
BL_NUM = [[0.0, 0.0, 1.0], [0.0, 0.0, -4.0, 10.0, -5.0]]
BL_DEN = [1.0, -2.0, 2.0]


def bl_f(p):
    return p * p / (p * p + (1 - p) ** 2)


def bl_g(p):
    return bl_f(p) * (1 - 5 * (1 - p) ** 2)


def spec_bl(n, scale, kl, scheme="A", rpoly=(), lattice=9):
    """Buckley-Leverett flux in lattice units: B = scale * (f, g)."""
    return dict(lattice=lattice, shape=(n, n), bc=["periodic"] * 3, scheme=scheme, d=1.0, s=[0.0] + [1.0] * 8,
                b=[[scale * v for v in BL_NUM[0]], [scale * v for v in BL_NUM[1]]], bden=BL_DEN,
                dpoly=[0.0, 1.0], dten=np.eye(3).tolist(), k0=(kl * np.eye(3)).tolist(), kpoly=[1.0],
                rpoly=list(rpoly), variant="remark3")


def test_numerators_are_eq54():
    x = np.linspace(0.0, 1.0, 11)
    q = np.polyval(BL_DEN[::-1], x)
    assert np.allclose(np.polyval(BL_NUM[0][::-1], x) / q, bl_f(x), rtol=1e-15, atol=1e-15)
    assert np.allclose(np.polyval(BL_NUM[1][::-1], x) / q, bl_g(x), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("scheme", ["A", "B"])
def test_common_factor_equals_polynomial_flux(scheme):
    rng = np.random.default_rng(41)
    phi0 = 0.5 + 0.1 * rng.uniform(-1, 1, (11, 13))
    base = dict(lattice=9, shape=(13, 11), bc=["periodic", "abb", "periodic"],
                phi_wall=[[0, 0], [0.3, 0.7], [0, 0]], scheme=scheme, d=1.0,
                s=[0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05], dpoly=[0.0, 1.0], dten=np.eye(3).tolist(),
                k0=[[0.02, 0.004, 0], [0.004, 0.015, 0], [0, 0, 0]], kpoly=[1.0, 0.0, 0.5],
                rpoly=[0.0, 0.01, -0.01] if scheme == "A" else [0.002], variant="remark3")
    cases = [  # (rational numerators, denominator) -> polynomial B
        (([0.0, 0.05, 0.05], [0.0, -0.03, -0.03]), [1.0, 1.0], ([0.0, 0.05], [0.0, -0.03])),
        (([0.0, 0.0, 0.2, 0.1], [0.0, 0.0, 0.1, 0.05]), [2.0, 1.0], ([0.0, 0.0, 0.1], [0.0, 0.0, 0.05])),
    ]
    for num, den, poly in cases:
        a = orc.run(orc.params_from_spec(dict(base, b=list(num), bden=den)), phi0, 40)[0]
        b = orc.run(orc.params_from_spec(dict(base, b=list(poly))), phi0, 40)[0]
        assert np.abs(a - phi0).max() > 1e-3
        assert np.abs(a - b).max() < 1e-14, np.abs(a - b).max()


def test_rational_flux_needs_remark3():
    sp = spec_bl(8, 0.1, 0.1)
    sp["variant"] = "standard"
    with pytest.raises(ValueError):
        orc.params_from_spec(sp)


def test_buckley_leverett_conserves_mass():
    n = 24
    x = (np.arange(n) + 0.5) / n * 3.0 - 1.5
    X, Y = np.meshgrid(x, x, indexing="xy")
    phi0 = np.where(X * X + Y * Y < 0.5, 1.0, 0.0)
    p = orc.params_from_spec(spec_bl(n, 0.1, 0.1))
    ph, _ = orc.run(p, phi0, 60)
    assert abs(ph.sum() - phi0.sum()) < 1e-12 * phi0.sum()
    assert np.abs(ph - phi0).max() > 1e-2


def _cstep(fn, p):
    """Derivative by complex step (Squire & Trapp 1998)."""
    h = 1e-30
    return np.imag(fn(p + 1j * h)) / h


def test_manufactured_solution_second_order():
    """phi = 0.5 + 0.25 sin(2 pi (x - t)) sin(2 pi y) on the periodic unit
    square solves Eq. 52 with the Buckley-Leverett f, g, kappa = 0.05 and
    R = d_t phi + f'(phi) d_x phi + g'(phi) d_y phi - kappa lap(phi), fed to
    Scheme B as an external source field (the f', g' here by complex step).
    Remark III runs with diffusive refinement (rates fixed) down to T = 0.2."""
    kappa, T = 0.05, 0.2
    gres = []
    for n in (32, 64, 128):
        dx = 1.0 / n
        dt = 0.16 * dx * dx / kappa            # lattice diffusivity 0.16 on every grid
        spec = spec_bl(n, dt / dx, kappa * dt / dx ** 2, scheme="B")
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")

        def exact(t):
            return 0.5 + 0.25 * np.sin(2 * math.pi * (X - t)) * np.sin(2 * math.pi * Y)

        def source(step):
            t = step * dt
            s1, c1 = np.sin(2 * math.pi * (X - t)), np.cos(2 * math.pi * (X - t))
            s2, c2 = np.sin(2 * math.pi * Y), np.cos(2 * math.pi * Y)
            ph = 0.5 + 0.25 * s1 * s2
            pt = -0.5 * math.pi * c1 * s2
            px = 0.5 * math.pi * c1 * s2
            py = 0.5 * math.pi * s1 * c2
            lap = -2 * (2 * math.pi) ** 2 * 0.25 * s1 * s2
            R = pt + _cstep(bl_f, ph) * px + _cstep(bl_g, ph) * py - kappa * lap
            return dt * R

        nst = int(round(T / dt))
        ph, _ = orc.run(orc.params_from_spec(spec), exact(0.0), nst, source=source)
        ex = exact(nst * dt)
        gres.append(float(np.abs(ph - ex).sum() / np.abs(ex).sum()))
    order = [math.log2(gres[i] / gres[i + 1]) for i in range(2)]
    print(f"Buckley-Leverett manufactured solution: GRE {gres}, orders {order}")
    assert all(1.7 <= o <= 2.3 for o in order), (gres, order)
