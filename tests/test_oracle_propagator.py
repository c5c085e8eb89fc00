"""Exact discrete propagator for linear periodic runs: a pin of the oracle's
relaxation with unequal rates.

With B = phi u, D = phi Dten, a constant K and no source, one step of Eq. 2
with the equilibrium of Eq. 3 is linear in the populations of a node:

    f^eq = w phi,  phi = 1^T f  (Eq. 10a),
    w_k  = omega_k [1 + c_k.u / cs^2 + (u u + d cs^2 Dten - cs^2 I):(c_k c_k - cs^2 I) / (2 cs^4)],
    f*   = L f,    L = I - M^-1 S M (I - w 1^T),

with S the diagonal rates of Eq. 17 and the flux block A = (K/(d cs^2) + I/2)^-1
of Eq. 26 on the rows of j_x, j_y (j_z).  Streaming f_k(x + c_k) = f*_k(x)
on a periodic grid is diagonal in Fourier space: for a wave number kappa,
f^(kappa, t + 1) = E(kappa) L f^(kappa, t) with E = diag(exp(-i kappa.c_k)).
The initial state of Eq. 40 is f^(kappa, 0) = w phi^0(kappa), so

    phi^(kappa, T) = 1^T (E L)^T w phi^0(kappa).

This file builds that map from the paper's own tables (Eq. 5, 6, 15, the
orthogonal D3Q19 basis of d'Humieres et al. 2002), numpy's matrix inverse,
FFT and matrix powers, and compares it with the oracle's time stepping, which
works node by node in velocity space with its own tables and inverse.  A rate
applied to the wrong moment row, a transposed A block, a wrong sign in Eq. 3
or a streaming direction error changes the result at the 1e-3 level or more.
"""
import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

CS2 = 1.0 / 3.0

# Eq. 5: D2Q9 velocities and weights
C9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
# Eq. 15 (c = 1): rows rho, e, eps, jx, qx, jy, qy, pxx, pxy
M9 = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
FLUX9 = (3, 5)

# Eq. 6: D3Q19 velocities (columns of the printed table) and weights
C19 = np.array([
    [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0],
    [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1],
]).T
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
FLUX19 = (3, 5, 7)


def m19():
    """The orthogonal polynomial basis of d'Humieres et al. (2002), rows
    (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz,
    mx, my, mz), evaluated on the velocities of Eq. 6."""
    x, y, z = (C19[:, a].astype(np.float64) for a in range(3))
    r2 = x * x + y * y + z * z
    rows = [np.ones(19), 19 * r2 - 30, (21 * r2 * r2 - 53 * r2 + 24) / 2,
            x, (5 * r2 - 9) * x, y, (5 * r2 - 9) * y, z, (5 * r2 - 9) * z,
            3 * x * x - r2, (3 * r2 - 5) * (3 * x * x - r2),
            y * y - z * z, (3 * r2 - 5) * (y * y - z * z),
            x * y, y * z, x * z,
            (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z]
    return np.array(rows)


def weq(c, w, u, d, dten):
    """w_k of f^eq = w phi for B = phi u, C = phi u u (Eq. 7 with C(0) = 0),
    D = phi Dten (Eq. 3)."""
    dim = c.shape[1]
    T = np.outer(u, u) + d * CS2 * dten - CS2 * np.eye(dim)
    out = np.empty(len(w))
    for k in range(len(w)):
        ck = c[k].astype(np.float64)
        out[k] = w[k] * (1 + ck @ u / CS2 + np.sum(T * (np.outer(ck, ck) - CS2 * np.eye(dim))) / (2 * CS2 * CS2))
    return out


def collision_matrix(M, flux, s, K, d):
    """Lambda = M^-1 S M with S of Eq. 17: diagonal rates, the flux block A of Eq. 26."""
    q = M.shape[0]
    S = np.diag(np.asarray(s[:q], dtype=np.float64))
    A = np.linalg.inv(K / (d * CS2) + 0.5 * np.eye(len(flux)))
    for i, a in enumerate(flux):
        for j, b in enumerate(flux):
            S[a, b] = A[i, j]
    return np.linalg.inv(M) @ S @ M


def propagate(c, w, M, flux, s, u, K, d, dten, phi0, T):
    """phi(T) of the linear periodic scheme by the exact Fourier propagator."""
    shape = phi0.shape                      # (ny, nx) or (nz, ny, nx)
    dim = c.shape[1]
    q = len(w)
    wv = weq(c, w, u, d, dten)
    Lam = collision_matrix(M, flux, s, K, d)
    L = np.eye(q) - Lam @ (np.eye(q) - np.outer(wv, np.ones(q)))
    # wave numbers per axis, in the array's axis order (x is the last axis)
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in shape], indexing="ij")
    kx = [ks[dim - 1 - a].reshape(-1) for a in range(dim)]         # kx[a]: component a (x, y, z)
    phase = sum(np.outer(kx[a], c[:, a]) for a in range(dim))      # [nk, q]
    E = np.exp(-1j * phase)
    G = E[:, :, None] * L[None, :, :]                              # E(kappa) L
    P = np.linalg.matrix_power(G, T)
    transfer = np.einsum("k,nkj,j->n", np.ones(q), P, wv)          # 1^T (E L)^T w
    out = np.fft.ifftn(transfer.reshape(shape) * np.fft.fftn(phi0))
    assert np.abs(out.imag).max() < 1e-10 * np.abs(out.real).max()
    return out.real


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _spec2(shape, s, u, K, d=1.0, dten=None):
    dt = np.eye(3) if dten is None else np.asarray(dten, dtype=np.float64)
    k3 = np.zeros((3, 3))
    k3[:2, :2] = K
    return dict(lattice=9, shape=shape, bc=["periodic"] * 3, scheme="A", d=d, s=list(s),
                b=[[0.0, u[0]], [0.0, u[1]]], dpoly=[0.0, 1.0], dten=dt.tolist(),
                k0=k3.tolist(), kpoly=[1.0], rpoly=[])


def test_propagator_c1_workload():
    """The linear Gaussian-hill workload as stated: 64 x 64, s1 = s2 = 1.2,
    u = (0.05, 0.02), kappa = 0.01, 1000 steps."""
    spec, phi0, T = W.hill_linear_64()
    _, ph = orc.run(orc.params_from_spec(spec), phi0, T, snapshots=(250, T))
    u = np.array(spec["b"][0][1:2] + spec["b"][1][1:2])
    K = np.asarray(spec["k0"])[:2, :2]
    for t in (250, T):
        want = propagate(C9, W9, M9, FLUX9, spec["s"], u, K, spec["d"], np.eye(2), phi0, t)
        err = rel_l2(ph[t], want)
        print(f"C1 step {t}: oracle vs propagator {err:.2e}")
        assert err <= 1e-13


def test_propagator_d2q9_all_rates_distinct():
    """Every non-flux rate different, full anisotropic K, d != 1, anisotropic
    D tensor, ragged periodic grid."""
    s = [0.0, 1.3, 1.1, 0.0, 1.4, 0.0, 0.9, 1.2, 1.05]
    u = np.array([0.07, -0.04])
    K = np.array([[0.02, 0.006], [0.006, 0.012]])
    dten = np.array([[1.0, 0.15, 0.0], [0.15, 0.85, 0.0], [0.0, 0.0, 1.0]])
    shape = (17, 24)
    spec = _spec2((24, 17), s, u, K, d=0.8, dten=dten)
    rng = np.random.default_rng(61)
    phi0 = 0.3 + rng.uniform(-1, 1, shape)
    T = 300
    got, _ = orc.run(orc.params_from_spec(spec), phi0, T)
    want = propagate(C9, W9, M9, FLUX9, s, u, K, 0.8, dten[:2, :2], phi0, T)
    err = rel_l2(got, want)
    print(f"D2Q9 distinct rates: oracle vs propagator {err:.2e}")
    assert err <= 1e-13
    # the pin is sensitive: exchanging two rates moves the result far beyond round-off
    s2 = list(s)
    s2[1], s2[2] = s2[2], s2[1]
    off = propagate(C9, W9, M9, FLUX9, s2, u, K, 0.8, dten[:2, :2], phi0, T)
    assert rel_l2(off, want) > 1e-6


def test_propagator_d3q19_unequal_rates():
    """D3Q19 on a periodic ragged grid with every non-flux rate different and
    a full K: the oracle's moment rows and rate slots against the basis and
    S of this file."""
    s = [0.0] + [1.0 + 0.04 * i for i in range(18)]
    u = np.array([0.03, -0.02, 0.01])
    K = W.random_spd3(17)
    shape = (7, 8, 9)                           # (nz, ny, nx)
    spec = W.spec_d3q19_aniso((9, 8, 7), K=K, u=tuple(u))
    spec["bc"] = ["periodic"] * 3
    spec["s"] = s
    rng = np.random.default_rng(62)
    phi0 = 0.5 + rng.uniform(-1, 1, shape)
    T = 60
    got, _ = orc.run(orc.params_from_spec(spec), phi0, T)
    want = propagate(C19, W19, m19(), FLUX19, s, u, K, 1.0, np.eye(3), phi0, T)
    err = rel_l2(got, want)
    print(f"D3Q19 unequal rates: oracle vs propagator {err:.2e}")
    assert err <= 1e-13


def test_propagator_tables_are_the_papers():
    """The tables of this file: Eq. 15 rows mutually orthogonal, flux rows equal
    to the velocity components, the D3Q19 basis orthogonal with rank 19, and
    the weights isotropic to second order."""
    for c, w, M, flux in ((C9, W9, M9, FLUX9), (C19, W19, m19(), FLUX19)):
        G = M @ M.T
        assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
        for a, r in enumerate(flux):
            assert np.array_equal(M[r], c[:, a])
        dim = c.shape[1]
        assert abs(w.sum() - 1) < 1e-15
        assert np.abs(np.einsum("k,ka,kb->ab", w, c, c) - CS2 * np.eye(dim)).max() < 1e-15


@pytest.mark.parametrize("q", [9, 19])
def test_propagator_conserves_and_reproduces_eq10(q):
    """Properties of L itself that the paper fixes: 1^T L = 1^T (collision
    conserves phi, Eq. 10a), and at kappa = 0 the mean of phi is unchanged."""
    if q == 9:
        c, w, M, flux = C9, W9, M9, FLUX9
        s, u, K = [0.0, 1.3, 1.1, 0, 1.4, 0, 0.9, 1.2, 1.05], np.array([0.07, -0.04]), np.array(
            [[0.02, 0.006], [0.006, 0.012]])
        dten = np.eye(2)
    else:
        c, w, M, flux = C19, W19, m19(), FLUX19
        s, u, K, dten = [0.0] + [1.0 + 0.04 * i for i in range(18)], np.array([0.03, -0.02, 0.01]), \
            W.random_spd3(17), np.eye(3)
    wv = weq(c, w, u, 1.0, dten)
    assert abs(wv.sum() - 1) < 1e-15                                # Eq. 10a
    assert np.abs(wv @ c - u).max() < 1e-15                         # Eq. 10b: sum c f^eq = B = phi u
    Lam = collision_matrix(M, flux, s, K, 1.0)
    L = np.eye(len(w)) - Lam @ (np.eye(len(w)) - np.outer(wv, np.ones(len(w))))
    assert np.abs(np.ones(len(w)) @ L - np.ones(len(w))).max() < 1e-14
