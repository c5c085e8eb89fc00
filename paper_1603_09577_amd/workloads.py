"""Problem descriptions and seeded synthetic inputs.

This module holds no arithmetic of the lattice Boltzmann method: it only
states problems in the form of the paper's Eq. 1 (polynomial coefficients of
B(phi), D(phi), K(phi) = K0 k(phi), R(phi), lattice, walls, rates) and draws
seeded initial fields.  The GPU binding and the CPU oracle each read these
plain dicts and derive every method quantity (C of Eq. 7, A of Eq. 26, the
equilibria, ...) on their own.

Lattice units throughout: node i of a periodic axis sits at x = i; node k of
an axis with anti-bounce-back walls sits at z = k + 1/2, walls at 0 and n.
"""
import numpy as np

__all__ = [
    "spec_linear_gaussian", "spec_nonlinear_2d", "spec_d3q19_aniso",
    "gaussian_hill", "noise_field", "gaussians_3d", "random_spd3",
    "hill_linear_64", "nonlinear_2d", "d3q19_walls", "adjoint_2d", "adjoint_2d_sourcefree", "batch_specs",
    "nonlinear_2d_walls_rates", "d3q19_walls_source",
    "burgers_fisher_wave", "spec_burgers_fisher",
]


def _rates(q, diag=1.0, **over):
    s = [float(diag)] * q
    s[0] = 0.0
    for k, v in over.items():
        s[int(k[1:])] = float(v)
    return s


# ----------------------------------------------------------------------------
# problem specs
# ----------------------------------------------------------------------------

def spec_linear_gaussian(n=64, u=(0.05, 0.02), kappa=0.01, s12=1.2, precision="f64"):
    """Linear isotropic CDE with constant velocity (Eq. 58/61 with K = kappa I):
    B = phi u, D = phi I, K = kappa I, R = 0.  Rates: s1 = s2 = s12, the other
    non-flux rates 1.0; the flux block follows from K."""
    return dict(
        lattice=9, shape=(n, n), bc=["periodic"] * 3, scheme="A", d=1.0,
        s=_rates(9, 1.0, s1=s12, s2=s12),
        b=[[0.0, u[0]], [0.0, u[1]]], dpoly=[0.0, 1.0], dten=np.eye(3).tolist(),
        k0=(kappa * np.eye(3)).tolist(), kpoly=[1.0], rpoly=[],
        precision=precision, phi_ref=0.0,
    )


# Grid spacing and time step of the nonlinear 2-D workloads, in the length and
# time units their coefficients are stated in.  Read with dx = dt = 1 the
# stated problem is linearly unstable on any grid (grid Peclet number
# |B'| dx / K_min of about 150); with dx = 1/32 and lattice speed
# c = dx / dt = 10 it is stable with flux relaxation rates between 1.0 and 1.7.
NONLINEAR_DX = 1.0 / 32.0
NONLINEAR_DT = NONLINEAR_DX / 10.0


def lattice_units(b, k0, rpoly, dx, dt):
    """Rewrite Eq. 1 with x' = x / dx, t' = t / dt: B' = B dt/dx, K' = K dt/dx^2,
    R' = R dt; D is unchanged.  Polynomials in phi keep their phi dependence."""
    cl = dt / dx
    b2 = [[v * cl for v in row] for row in b]
    k2 = (np.asarray(k0, dtype=np.float64) * dt / (dx * dx)).tolist()
    r2 = [v * dt for v in rpoly]
    return b2, k2, r2


def spec_nonlinear_2d(nx=1024, ny=None, bcoef=0.5, k0=((0.02, 0.008), (0.008, 0.01)),
                      source=True, precision="f64", phi_ref=0.5,
                      dx=NONLINEAR_DX, dt=NONLINEAR_DT):
    """Nonlinear anisotropic CDE with source: B = bcoef phi^2 (1, 1),
    K = K0 (1 + phi^2), D = phi I, R = 0.1 phi (1 - phi) (or 0), Scheme A,
    on a periodic nx x ny grid of spacing dx, time step dt (coefficients
    returned in lattice units)."""
    ny = nx if ny is None else ny
    k = np.zeros((3, 3))
    k[:2, :2] = np.asarray(k0, dtype=np.float64)
    b, kl, r = lattice_units([[0.0, 0.0, bcoef], [0.0, 0.0, bcoef]], k,
                             [0.0, 0.1, -0.1] if source else [], dx, dt)
    return dict(
        lattice=9, shape=(nx, ny), bc=["periodic"] * 3, scheme="A", d=1.0,
        s=_rates(9, 1.0),
        b=b, dpoly=[0.0, 1.0], dten=np.eye(3).tolist(),
        k0=kl, kpoly=[1.0, 0.0, 1.0], rpoly=r,
        precision=precision, phi_ref=phi_ref,
    )


def spec_d3q19_aniso(n=(256, 256, 256), K=None, u=(0.03, 0.0, 0.01), phi_wall=0.0,
                     precision="f64", phi_ref=0.0, s_other=1.0):
    """Linear anisotropic CDE on D3Q19: B = phi u, D = phi I, constant full K,
    periodic in x and y, anti-bounce-back Dirichlet walls at both z ends."""
    if K is None:
        K = random_spd3(3)
    return dict(
        lattice=19, shape=tuple(n), bc=["periodic", "periodic", "abb"],
        phi_wall=[[0.0, 0.0], [0.0, 0.0], [phi_wall, phi_wall]], scheme="A", d=1.0,
        s=_rates(19, s_other),
        b=[[0.0, u[0]], [0.0, u[1]], [0.0, u[2]]], dpoly=[0.0, 1.0], dten=np.eye(3).tolist(),
        k0=np.asarray(K).tolist(), kpoly=[1.0], rpoly=[],
        precision=precision, phi_ref=phi_ref,
    )


def burgers_fisher_wave(y, t, a=4.0, b=1.0, kappa=0.4, delta=1.0, y0=0.0):
    """Travelling-wave solution of the Burgers-Fisher equation (Sec. 3.2,
    Eq. 46) reduced to one dimension along y,
        d_t phi + a phi^delta d_y phi = kappa d_yy phi + b phi (1 - phi^delta),
    phi = {1/2 + 1/2 tanh[A (y - y0 - omega t)]}^(1/delta) with
        A = -a delta / (2 kappa (delta + 1)),
        omega = (a^2 + b kappa (delta + 1)^2) / (a (delta + 1)),
    obtained by substituting the form of Eq. 47 into the one-dimensional
    equation (Eq. 48 is the same with x + y, whose diffusivity is 2 kappa; the
    tests check this form by substitution)."""
    A = -a * delta / (2.0 * kappa * (delta + 1.0))
    om = (a * a + b * kappa * (delta + 1.0) ** 2) / (a * (delta + 1.0))
    return (0.5 + 0.5 * np.tanh(A * (np.asarray(y, dtype=np.float64) - y0 - om * t))) ** (1.0 / delta)


def spec_burgers_fisher(n, nx=2, a=4.0, b=1.0, kappa=0.4, length=3.0, klat=0.1, precision="f64",
                        scheme="A"):
    """D2Q9 problem of the Burgers-Fisher wave along y (delta = 1): B = (0,
    a/2 phi^2) (Eq. 49 turned onto y), K = kappa I, D = phi I (Eq. 51),
    R = b phi (1 - phi) (Eq. 46), anti-bounce-back walls half a link beyond
    the first and last of n nodes on an axis of `length`, periodic in x (nx
    nodes; the solution does not depend on x).  Diffusive scaling: the lattice
    diffusivity is klat on every grid, dx = length / n, dt = klat dx^2 / kappa.
    Returns (spec in lattice units, dx, dt); the wall values are set from
    burgers_fisher_wave by the caller, per step."""
    dx = length / n
    dt = klat * dx * dx / kappa
    spec = dict(lattice=9, shape=(nx, n), bc=["periodic", "abb", "periodic"],
                phi_wall=[[0.0, 0.0], [0.0, 0.0], [0.0, 0.0]], scheme=scheme, d=1.0, s=_rates(9, 1.0),
                b=[[0.0], [0.0, 0.0, 0.5 * a * dt / dx]], dpoly=[0.0, 1.0], dten=np.eye(3).tolist(),
                k0=(klat * np.eye(3)).tolist(), kpoly=[1.0], rpoly=[0.0, b * dt, -b * dt],
                precision=precision, phi_ref=0.5)
    return spec, dx, dt


# ----------------------------------------------------------------------------
# seeded fields
# ----------------------------------------------------------------------------

def gaussian_hill(n=64, sigma0=6.0, centre=None, amp=1.0, images=2):
    """Gaussian hill of amplitude ``amp`` and width sigma0 on an n x n periodic
    grid, summed over periodic images |i|,|j| <= images.  Returns [ny, nx]."""
    centre = (n / 2.0, n / 2.0) if centre is None else centre
    x = np.arange(n, dtype=np.float64)
    X, Y = np.meshgrid(x, x, indexing="xy")
    out = np.zeros((n, n))
    for i in range(-images, images + 1):
        for j in range(-images, images + 1):
            dx = X - centre[0] - i * n
            dy = Y - centre[1] - j * n
            out += np.exp(-(dx * dx + dy * dy) / (2.0 * sigma0 * sigma0))
    return amp * out


def noise_field(shape, seed, mean=0.5, amp=0.1):
    """mean + amp * U[-1, 1) from numpy's PCG64 generator, C order."""
    rng = np.random.default_rng(seed)
    return mean + amp * rng.uniform(-1.0, 1.0, size=shape)


def random_spd3(seed, lo=0.005, hi=0.05):
    """Symmetric 3x3 tensor Q diag(lam) Q^T, Q from the QR of a seeded normal
    matrix (signs fixed so that diag(R) > 0), lam ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(R))[None, :]
    lam = rng.uniform(lo, hi, size=3)
    K = Q @ np.diag(lam) @ Q.T
    return 0.5 * (K + K.T)


def gaussians_3d(n=(256, 256, 256), seed=3, count=8):
    """Sum of ``count`` Gaussians: amplitude U[0.5, 1], width U[8, 24] cells
    (scaled with the grid), centres uniform in x, y and in the middle 69% of z;
    periodic images in x and y.  Node k of z sits at k + 1/2.  Returns [nz, ny, nx]."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    scale = min(nx, ny, nz) / 256.0
    amp = rng.uniform(0.5, 1.0, size=count)
    sig = rng.uniform(8.0, 24.0, size=count) * scale
    cx = rng.uniform(0, nx, size=count)
    cy = rng.uniform(0, ny, size=count)
    cz = rng.uniform(40.0 / 256.0 * nz, 216.0 / 256.0 * nz, size=count)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64) + 0.5
    out = np.zeros((nz, ny, nx))
    for g in range(count):
        gz = np.exp(-((z - cz[g]) ** 2) / (2 * sig[g] ** 2))
        gy = np.zeros(ny)
        gx = np.zeros(nx)
        for i in (-1, 0, 1):
            gy += np.exp(-((y - cy[g] - i * ny) ** 2) / (2 * sig[g] ** 2))
            gx += np.exp(-((x - cx[g] - i * nx) ** 2) / (2 * sig[g] ** 2))
        out += amp[g] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return out


# ----------------------------------------------------------------------------
# the five workloads (plus the non-degenerate gradient variant)
# ----------------------------------------------------------------------------

def hill_linear_64():
    """D2Q9, linear isotropic CDE, periodic 64 x 64, u = (0.05, 0.02),
    kappa = 0.01, Gaussian hill (amplitude 1, sigma 6, centred), R = 0,
    s1 = s2 = 1.2, 1000 steps."""
    spec = spec_linear_gaussian(64)
    return spec, gaussian_hill(64, 6.0), 1000


def nonlinear_2d(n=1024, precision="f64"):
    """D2Q9 nonlinear anisotropic CDE, periodic n x n, phi0 = 0.5 + 0.1 U[-1, 1)
    (seed 2), Scheme A source, 5000 steps."""
    spec = spec_nonlinear_2d(n, precision=precision)
    return spec, noise_field((n, n), 2), 5000


def d3q19_walls(n=(256, 256, 256), precision="f64"):
    """D3Q19 anisotropic CDE, periodic x/y, phi_w = 0 walls on z, K from seed 3,
    u = (0.03, 0, 0.01), sum of 8 Gaussians (seed 3), 2000 steps."""
    spec = spec_d3q19_aniso(n, K=random_spd3(3), precision=precision, phi_ref=0.0)
    return spec, gaussians_3d(n, 3), 2000


def nonlinear_2d_walls_rates(n=1024, precision="f64"):
    """The nonlinear 2-D physics between anti-bounce-back walls on y (phi_w =
    0.3 below, 0.7 above) with unequal non-flux rates, seed 5, 5000 steps."""
    spec = spec_nonlinear_2d(n, precision=precision)
    spec = dict(spec, bc=["periodic", "abb", "periodic"], phi_wall=[[0.0, 0.0], [0.3, 0.7], [0.0, 0.0]],
                s=[0.0, 1.3, 1.1, 1.0, 1.4, 1.0, 0.9, 1.2, 1.05])
    return spec, noise_field((n, n), 5), 5000


def d3q19_walls_source(n=(128, 128, 128), precision="f64"):
    """The D3Q19 walls workload with a Scheme-A source R = 0.002 - 0.004 phi +
    0.001 phi^2 (R' < 0 on the range phi takes, so perturbations decay rather
    than grow; the root at phi = 2 - sqrt(2) attracts) and K = K0 (1 + phi^2 /
    2), 1000 steps."""
    spec, phi0, _ = d3q19_walls(n, precision=precision)
    spec = dict(spec, rpoly=[0.002, -0.004, 0.001], kpoly=[1.0, 0.0, 0.5])
    return spec, phi0, 1000


def adjoint_2d(n=512, precision="f64"):
    """Adjoint workload: the nonlinear 2-D physics on n x n (seed 5), target phi* from seed 6,
    2000 steps, sqrt(T) = 45-step checkpoints."""
    spec = spec_nonlinear_2d(n, precision=precision)
    return spec, noise_field((n, n), 5), noise_field((n, n), 6), 2000


def adjoint_2d_sourcefree(n=512, precision="f64", nsteps=2000):
    """Non-degenerate gradient variant of the adjoint workload: R = 0, so the sensitivities do
    not vanish; the target is a forward run of the same model from seed 6."""
    spec = spec_nonlinear_2d(n, precision=precision, source=False)
    return spec, noise_field((n, n), 5), noise_field((n, n), 6), nsteps


def batch_specs(count=512, seed=4, lo=32, hi=512, precision="f32"):
    """Batched workload: ``count`` independent D2Q9 instances, sides uniform in
    [lo, hi] (square with probability 1/2), per-instance K0 = Rot diag(lam)
    Rot^T with lam ~ U[0.005, 0.05], B = c phi^2 (1, 1) with c ~ U[0, 1],
    K = K0 (1 + phi^2), R = 0, phi0 = 0.15 + 0.05 U[-1, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(rng.integers(lo, hi + 1))
        ny = nx if rng.uniform() < 0.5 else int(rng.integers(lo, hi + 1))
        th = rng.uniform(0.0, np.pi)
        lam = rng.uniform(0.005, 0.05, size=2)
        Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        K0 = Rm @ np.diag(lam) @ Rm.T
        c = rng.uniform(0.0, 1.0)
        spec = spec_nonlinear_2d(nx, ny, bcoef=c, k0=0.5 * (K0 + K0.T), source=False,
                                 precision=precision, phi_ref=0.15)
        phi0 = noise_field((ny, nx), seed * 100003 + i, mean=0.15, amp=0.05)
        out.append((spec, phi0))
    return out
