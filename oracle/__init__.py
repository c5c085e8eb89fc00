"""Python access to the CPU FP64 oracle (ctypes over oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path (the GPU library
and its binding) never imports it, and the oracle imports nothing from the
product.  A problem is described by a plain dict (see ``params_from_spec``);
both sides read the same dict and derive every method quantity themselves.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAXP = 9

_lib = None


class Params(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc", ctypes.c_int * 3),
        ("phi_wall", (ctypes.c_double * 2) * 3),
        ("scheme", ctypes.c_int),
        ("d", ctypes.c_double),
        ("s", ctypes.c_double * 19),
        ("basis", ctypes.c_int),
        ("bpoly", (ctypes.c_double * MAXP) * 3),
        ("dpoly", ctypes.c_double * MAXP),
        ("dten", (ctypes.c_double * 3) * 3),
        ("k0", (ctypes.c_double * 3) * 3),
        ("kpoly", ctypes.c_double * MAXP),
        ("rpoly", ctypes.c_double * MAXP),
        ("variant", ctypes.c_int),
        ("bden", ctypes.c_double * MAXP),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_P = ctypes.POINTER(Params)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_check.argtypes = [_P]
        L.orc_check.restype = ctypes.c_int
        L.orc_tables.argtypes = [_P, _I, _D, _D, _D]
        L.orc_ctensor.argtypes = [_P, ctypes.c_double, _D]
        L.orc_feq.argtypes = [_P, ctypes.c_double, _D]
        L.orc_ablock.argtypes = [_P, ctypes.c_double, _D, _D]
        L.orc_collide.argtypes = [_P, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc_init.argtypes = [_P, _D, _D, _D, _D]
        L.orc_step.argtypes = [_P, _D, _D, _D, _D, _D, ctypes.c_int]
        L.orc_step.restype = ctypes.c_int
        L.orc_phi.argtypes = [_P, _D, _D, _D]
        L.orc_adjoint_step.argtypes = [_P, _D, _D, _D, _D, _D, _D, _D, _D, _D, ctypes.c_int]
        L.orc_adjoint_init.argtypes = [_P, _D, _D, _D, _D, _D]
        L.orc_node_jacobian.argtypes = [_P, _D, ctypes.c_double, _D]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _pad(coeffs, n=MAXP):
    out = [0.0] * n
    for i, c in enumerate(coeffs or []):
        out[i] = float(c)
    return out


BC_CODES = {"periodic": 0, "abb": 1}


def params_from_spec(spec, basis=0):
    """Oracle parameter block from a problem dict.

    Keys: lattice (9 | 19), shape (nx, ny[, nz]), bc (per axis "periodic" |
    "abb"), phi_wall ([[lo, hi]] * 3), scheme ("A" | "B"), d, s (rates in
    moment-row order), b (per axis polynomial coefficients of B), dpoly, dten,
    k0, kpoly, rpoly, variant ("standard" | "remark3": Eq. 36-38), bden
    (denominator of a rational B = b / bden, Remark III only; default 1).
    """
    p = Params()
    q = int(spec["lattice"])
    p.q = q
    shape = list(spec["shape"]) + [1] * (3 - len(spec["shape"]))
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    bc = list(spec.get("bc", ["periodic"] * 3)) + ["periodic"] * 3
    for a in range(3):
        p.bc[a] = BC_CODES[bc[a]]
    pw = spec.get("phi_wall", [[0.0, 0.0]] * 3)
    for a in range(3):
        p.phi_wall[a][0] = float(pw[a][0])
        p.phi_wall[a][1] = float(pw[a][1])
    p.scheme = {"A": 0, "B": 1}[spec.get("scheme", "A")]
    p.variant = {"standard": 0, "remark3": 1}[spec.get("variant", "standard")]
    p.d = float(spec.get("d", 1.0))
    s = _pad(spec["s"], 19)
    for i in range(19):
        p.s[i] = s[i]
    p.basis = basis
    b = spec["b"]
    for a in range(3):
        row = _pad(b[a] if a < len(b) else [])
        for i in range(MAXP):
            p.bpoly[a][i] = row[i]
    for name in ("dpoly", "kpoly", "rpoly"):
        row = _pad(spec.get(name, {"dpoly": [0, 1], "kpoly": [1], "rpoly": []}[name]))
        arr = getattr(p, name)
        for i in range(MAXP):
            arr[i] = row[i]
    row = _pad(spec.get("bden", []))
    for i in range(MAXP):
        p.bden[i] = row[i]
    dten = np.asarray(spec.get("dten", np.eye(3)), dtype=np.float64)
    k0 = np.asarray(spec["k0"], dtype=np.float64)
    for a in range(3):
        for c in range(3):
            p.dten[a][c] = dten[a, c] if a < dten.shape[0] and c < dten.shape[1] else 0.0
            p.k0[a][c] = k0[a, c] if a < k0.shape[0] and c < k0.shape[1] else 0.0
    rc = lib().orc_check(ctypes.byref(p))
    if rc != 0:
        raise ValueError(f"oracle rejects the parameter set (code {rc})")
    return p


def nodes(p):
    return p.nx * p.ny * p.nz


def field_shape(p):
    return (p.nz, p.ny, p.nx) if p.q == 19 else (p.ny, p.nx)


def tables(p):
    q = p.q
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    M = np.zeros((q, q))
    Minv = np.zeros((q, q))
    lib().orc_tables(ctypes.byref(p), c.ctypes.data_as(_I), _ptr(w), _ptr(M), _ptr(Minv))
    return c, w, M, Minv


def ctensor(p, phi):
    out = np.zeros(9)
    lib().orc_ctensor(ctypes.byref(p), float(phi), _ptr(out))
    return out.reshape(3, 3)


def feq(p, phi):
    out = np.zeros(p.q)
    lib().orc_feq(ctypes.byref(p), float(phi), _ptr(out))
    return out


def ablock(p, phi, kloc=None):
    dim = 2 if p.q == 9 else 3
    out = np.zeros(dim * dim)
    kl = None if kloc is None else np.ascontiguousarray(kloc, dtype=np.float64).reshape(9)
    lib().orc_ablock(ctypes.byref(p), float(phi), _ptr(kl), _ptr(out))
    return out.reshape(dim, dim)


def collide(p, f, pprev=None, rext=0.0, rext_prev=0.0, kloc=None):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(p.q)
    phi = ctypes.c_double()
    if pprev is None:
        pprev = float(f.sum())
    kl = None if kloc is None else np.ascontiguousarray(kloc, dtype=np.float64).reshape(9)
    lib().orc_collide(ctypes.byref(p), _ptr(f), float(pprev), float(rext), float(rext_prev),
                      _ptr(kl), _ptr(out), ctypes.byref(phi))
    return out, phi.value


def init(p, phi0, rext0=None):
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
    N = nodes(p)
    assert phi0.size == N
    f = np.zeros(p.q * N)
    pp = np.zeros(N)
    r0 = None if rext0 is None else np.ascontiguousarray(rext0, dtype=np.float64).reshape(-1)
    lib().orc_init(ctypes.byref(p), _ptr(phi0), _ptr(r0), _ptr(f), _ptr(pp))
    return f, pp


def step(p, f, pp, rext=None, rext_prev=None, kfield=None, nthreads=0):
    """One time step in place on (f, pp)."""
    r = None if rext is None else np.ascontiguousarray(rext, dtype=np.float64).reshape(-1)
    rp = None if rext_prev is None else np.ascontiguousarray(rext_prev, dtype=np.float64).reshape(-1)
    kf = None if kfield is None else np.ascontiguousarray(kfield, dtype=np.float64).reshape(-1)
    rc = lib().orc_step(ctypes.byref(p), _ptr(f), _ptr(pp), _ptr(r), _ptr(rp), _ptr(kf), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_step failed ({rc})")


def phi(p, f, rext=None):
    out = np.zeros(nodes(p))
    r = None if rext is None else np.ascontiguousarray(rext, dtype=np.float64).reshape(-1)
    lib().orc_phi(ctypes.byref(p), _ptr(f), _ptr(r), _ptr(out))
    return out.reshape(field_shape(p))


def run(p, phi0, nsteps, snapshots=(), nthreads=0, source=None, kfield=None):
    """Run nsteps from phi0.  ``source(t)`` (optional) returns the external
    field R(x, t).  Returns (phi(nsteps), {t: phi(t) for t in snapshots})."""
    r0 = None if source is None else source(0)
    f, pp = init(p, phi0, r0)
    snaps = {}
    if 0 in snapshots:
        snaps[0] = phi(p, f, r0)
    rprev = r0
    for t in range(nsteps):
        rt = None if source is None else source(t)
        step(p, f, pp, rt, rprev if source is not None else None, kfield, nthreads)
        rprev = rt
        if (t + 1) in snapshots:
            snaps[t + 1] = phi(p, f, None if source is None else source(t + 1))
    return phi(p, f, None if source is None else source(nsteps)), snaps


def node_jacobian(p, f, pprev):
    q = p.q
    jac = np.zeros((q + 1) * (q + 7))
    f = np.ascontiguousarray(f, dtype=np.float64)
    lib().orc_node_jacobian(ctypes.byref(p), _ptr(f), float(pprev), _ptr(jac))
    return jac.reshape(q + 1, q + 7)


def adjoint_step(p, f, pp, lam_next, mu_next, nthreads=0):
    N = nodes(p)
    lam = np.zeros(p.q * N)
    mu = np.zeros(N)
    gk = np.zeros(9)
    lib().orc_adjoint_step(ctypes.byref(p), _ptr(f), _ptr(pp), _ptr(lam_next), _ptr(mu_next),
                           None, None, _ptr(lam), _ptr(mu), _ptr(gk), int(nthreads))
    return lam, mu, gk.reshape(3, 3)


def adjoint_init(p, phi0, lam0, mu0):
    g = np.zeros(nodes(p))
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
    lib().orc_adjoint_init(ctypes.byref(p), _ptr(phi0), None, _ptr(lam0), _ptr(mu0), _ptr(g))
    return g.reshape(field_shape(p))


def gradient(p, phi0, nsteps, dl_dphi, nthreads=0):
    """Discrete adjoint of a run: returns (phi(T), dL/dphi0, dL/dK0) where
    ``dl_dphi(phiT)`` gives dL/dphi(T).  dL/dK0 is returned for the symmetric
    parametrisation (xx, xy, yy[, xz, yz, zz]) as a dict.  Stores every state;
    small problems only."""
    f, pp = init(p, phi0)
    states = []
    for _ in range(nsteps):
        states.append((f.copy(), pp.copy()))
        step(p, f, pp, nthreads=nthreads)
    phiT = phi(p, f)
    g = np.ascontiguousarray(dl_dphi(phiT), dtype=np.float64).reshape(-1)
    N = nodes(p)
    lam = np.tile(g, p.q)           # dphi/df_k = 1 for every k
    mu = np.zeros(N)
    gk = np.zeros((3, 3))
    for t in range(nsteps - 1, -1, -1):
        fs, ps = states[t]
        lam, mu, g_t = adjoint_step(p, fs, ps, lam, mu, nthreads)
        gk += g_t
    gphi0 = adjoint_init(p, phi0, lam, mu)
    gk_named = {"xx": gk[0, 0], "xy": gk[0, 1], "yy": gk[1, 1]}
    if p.q == 19:
        gk_named.update({"xz": gk[0, 2], "yz": gk[1, 2], "zz": gk[2, 2]})
    return phiT, gphi0, gk_named
