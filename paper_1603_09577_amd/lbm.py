"""Thin ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory and the stream.  Importing
this module does not load the library; the first call does, and raises
``LbmLibraryMissing`` if it has not been built (python -m
paper_1603_09577_amd.build).  There is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PAPER_LBM_LIB selects another build of the same library (e.g. a variant)
LIB_PATH = os.environ.get("PAPER_LBM_LIB") or os.path.join(HERE, "liblbm.so")
MAXP = 9

LBM_OK, LBM_E_INVALID, LBM_E_UNSUPPORTED, LBM_E_HIP, LBM_E_DIVERGED, LBM_E_STATE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"f64": 0, "f32": 1, "f16": 2}
FLAG_MOMENT_PATH = 1
FLAG_NO_XCD_REMAP = 2
FLAG_NO_GRAPH = 4
FLAG_REMARK3 = 8

# every symbol include/lbm.h declares
EXPORTS = [
    "lbm_create", "lbm_state_bytes", "lbm_adjoint_bytes", "lbm_init", "lbm_step", "lbm_sweep", "lbm_get_phi",
    "lbm_phi_of", "lbm_current", "lbm_set_current", "lbm_set_check", "lbm_set_k0",
    "lbm_reduce", "lbm_adjoint_seed", "lbm_adjoint_step", "lbm_adjoint_init",
    "lbm_adjoint_grad_k0", "lbm_destroy", "lbm_last_error",
    "lbm_batch_create", "lbm_batch_layout", "lbm_batch_instance", "lbm_batch_init",
    "lbm_batch_step", "lbm_batch_get_phi", "lbm_batch_tune", "lbm_batch_set_shape",
    "lbm_batch_get_shape", "lbm_batch_destroy", "lbm_probe_copy", "lbm_set_chunk", "lbm_tune",
    "lbm_set_nontemporal", "lbm_recenter", "lbm_set_recenter", "lbm_set_fields", "lbm_set_phi_wall",
    "lbm_set_two_step", "lbm_two_step_shape", "lbm_adjoint_step2", "lbm_adjoint_pair_ok", "lbm_set_remap",
    "lbm_adjoint_tile_shape", "lbm_set_adjoint_tile", "lbm_adjoint_tile",
    "lbm_reduce_async", "lbm_reduce_state", "lbm_reduce_noalloc",
]


class LbmLibraryMissing(RuntimeError):
    pass


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


class LbmDesc(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc", ctypes.c_int * 3),
        ("phi_wall", (ctypes.c_double * 2) * 3),
        ("precision", ctypes.c_int),
        ("phi_ref", ctypes.c_double),
        ("scheme", ctypes.c_int),
        ("d", ctypes.c_double),
        ("s", ctypes.c_double * 19),
        ("b", (ctypes.c_double * MAXP) * 3),
        ("dpoly", ctypes.c_double * MAXP),
        ("dten", (ctypes.c_double * 3) * 3),
        ("k0", (ctypes.c_double * 3) * 3),
        ("kpoly", ctypes.c_double * MAXP),
        ("rpoly", ctypes.c_double * MAXP),
        ("flags", ctypes.c_int),
        ("plane_pad", ctypes.c_int),
        ("bden", ctypes.c_double * MAXP),
    ]


_lib = None
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)


def load():
    """Load liblbm.so (raises LbmLibraryMissing when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LbmLibraryMissing(
            f"{LIB_PATH} not found: build it with `python -m paper_1603_09577_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "lbm_create": ([ctypes.POINTER(LbmDesc), ctypes.POINTER(_VP)], ctypes.c_int),
        "lbm_state_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                             ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_adjoint_bytes": ([_VP, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_init": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_step": ([_VP, ctypes.c_int, _VP], ctypes.c_int),
        "lbm_sweep": ([_VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_get_phi": ([_VP, _VP, _VP], ctypes.c_int),
        "lbm_phi_of": ([_VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_current": ([_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
        "lbm_set_current": ([_VP, ctypes.c_int, ctypes.c_longlong], ctypes.c_int),
        "lbm_set_check": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_set_k0": ([_VP, _DP], ctypes.c_int),
        "lbm_reduce": ([_VP, _VP, _VP, _DP, _VP], ctypes.c_int),
        "lbm_adjoint_seed": ([_VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_adjoint_step": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_adjoint_init": ([_VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_adjoint_grad_k0": ([_VP, _DP, _VP], ctypes.c_int),
        "lbm_destroy": ([_VP], None),
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_batch_create": ([ctypes.POINTER(LbmDesc), ctypes.c_int, ctypes.POINTER(_VP)], ctypes.c_int),
        "lbm_batch_layout": ([_VP, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
        "lbm_batch_instance": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "lbm_batch_init": ([_VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_batch_step": ([_VP, ctypes.c_int, _VP], ctypes.c_int),
        "lbm_batch_get_phi": ([_VP, _VP, _VP], ctypes.c_int),
        "lbm_batch_tune": ([_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
        "lbm_batch_set_shape": ([_VP, ctypes.c_int, ctypes.c_uint, ctypes.c_int], ctypes.c_int),
        "lbm_batch_get_shape": ([_VP, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "lbm_batch_destroy": ([_VP], None),
        "lbm_probe_copy": ([_VP, _VP, ctypes.c_size_t, ctypes.c_int, _VP], ctypes.c_int),
        "lbm_set_chunk": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_set_nontemporal": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_tune": ([_VP, ctypes.c_int, _VP, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
        "lbm_recenter": ([_VP, _VP], ctypes.c_int),
        "lbm_set_recenter": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_set_fields": ([_VP, _VP, _VP], ctypes.c_int),
        "lbm_set_phi_wall": ([_VP, ctypes.c_double, ctypes.c_double, _VP], ctypes.c_int),
        "lbm_set_two_step": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_set_remap": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_two_step_shape": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                               ctypes.c_int),
        "lbm_adjoint_step2": ([_VP] * 10, ctypes.c_int),
        "lbm_adjoint_pair_ok": ([_VP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "lbm_adjoint_tile_shape": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                                   ctypes.c_int),
        "lbm_set_adjoint_tile": ([_VP, ctypes.c_int], ctypes.c_int),
        "lbm_adjoint_tile": ([_VP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "lbm_reduce_async": ([_VP, _VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_reduce_state": ([_VP, _VP, _VP, _VP], ctypes.c_int),
        "lbm_reduce_noalloc": ([_VP, _VP, ctypes.c_size_t, _VP, _VP], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error().decode())


def _pad(coeffs, n=MAXP):
    out = [0.0] * n
    for i, c in enumerate(coeffs or []):
        out[i] = float(c)
    return out


def desc_from_spec(spec, flags=0):
    """lbm_desc from a problem dict (see paper_1603_09577_amd.workloads)."""
    d = LbmDesc()
    d.lattice = int(spec["lattice"])
    shape = list(spec["shape"]) + [1] * (3 - len(spec["shape"]))
    d.nx, d.ny, d.nz = (int(v) for v in shape)
    bc = list(spec.get("bc", ["periodic"] * 3)) + ["periodic"] * 3
    for a in range(3):
        d.bc[a] = {"periodic": 0, "abb": 1}[bc[a]]
    pw = spec.get("phi_wall", [[0.0, 0.0]] * 3)
    for a in range(3):
        d.phi_wall[a][0], d.phi_wall[a][1] = float(pw[a][0]), float(pw[a][1])
    d.precision = PRECISIONS[spec.get("precision", "f64")]
    d.phi_ref = float(spec.get("phi_ref", 0.0))
    d.scheme = {"A": 0, "B": 1}[spec.get("scheme", "A")]
    d.d = float(spec.get("d", 1.0))
    s = _pad(spec["s"], 19)
    for i in range(19):
        d.s[i] = s[i]
    b = spec["b"]
    for a in range(3):
        row = _pad(b[a] if a < len(b) else [])
        for i in range(MAXP):
            d.b[a][i] = row[i]
    for name, default in (("dpoly", [0.0, 1.0]), ("kpoly", [1.0]), ("rpoly", [])):
        row = _pad(spec.get(name, default))
        arr = getattr(d, name)
        for i in range(MAXP):
            arr[i] = row[i]
    dten = np.asarray(spec.get("dten", np.eye(3)), dtype=np.float64)
    k0 = np.asarray(spec["k0"], dtype=np.float64)
    for a in range(3):
        for c in range(3):
            d.dten[a][c] = dten[a, c] if a < dten.shape[0] and c < dten.shape[1] else 0.0
            d.k0[a][c] = k0[a, c] if a < k0.shape[0] and c < k0.shape[1] else 0.0
    d.flags = int(flags | spec.get("flags", 0) | (FLAG_REMARK3 if spec.get("variant") == "remark3" else 0))
    d.plane_pad = int(spec.get("plane_pad", 0))
    row = _pad(spec.get("bden", []))
    for i in range(MAXP):
        d.bden[i] = row[i]
    return d


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Lbm:
    """One MRT lattice Boltzmann instance on the current GPU.

    Owns two distribution buffers, the phi-history buffer and, where two
    steps per pass read one, the second history buffer as torch tensors (uint8
    storage, sizes from lbm_state_bytes), and the library context.
    """

    def __init__(self, spec, device="cuda", flags=0):
        import torch
        self.spec = spec
        self.lib = load()
        self.desc = desc_from_spec(spec, flags)
        ctx = _VP()
        _check(self.lib.lbm_create(ctypes.byref(self.desc), ctypes.byref(ctx)))
        self.ctx = ctx
        fb, pb, p2b = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(self.lib.lbm_state_bytes(self.ctx, ctypes.byref(fb), ctypes.byref(pb), ctypes.byref(p2b)))
        self.f_bytes, self.p_bytes, self.p2_bytes = fb.value, pb.value, p2b.value
        self.device = torch.device(device)
        self.shape = (self.desc.nz, self.desc.ny, self.desc.nx) if self.desc.lattice == 19 \
            else (self.desc.ny, self.desc.nx)
        self.q = self.desc.lattice
        self.N = int(np.prod(self.shape))
        self.f = [torch.empty(self.f_bytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.p = torch.empty(self.p_bytes, dtype=torch.uint8, device=self.device)
        self.p2 = torch.empty(self.p2_bytes, dtype=torch.uint8, device=self.device) if self.p2_bytes else None
        self.compute_dtype = torch.float64 if self.desc.precision == 0 else torch.float32

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.lbm_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- forward -----------------------------------------------------------
    def init(self, phi0, stream=None):
        import torch
        phi0 = torch.as_tensor(phi0, dtype=torch.float64, device=self.device).contiguous()
        assert phi0.numel() == self.N
        self._phi0 = phi0
        _check(self.lib.lbm_init(self.ctx, _ptr(phi0), _ptr(self.f[0]), _ptr(self.f[1]), _ptr(self.p),
                                 _ptr(self.p2), _stream(stream)))
        return self

    def step(self, n=1, stream=None):
        _check(self.lib.lbm_step(self.ctx, int(n), _stream(stream)))

    def sweep(self, f_in, f_out, p, stream=None):
        _check(self.lib.lbm_sweep(self.ctx, _ptr(f_in), _ptr(f_out), _ptr(p), _stream(stream)))

    def phi(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(self.lib.lbm_get_phi(self.ctx, _ptr(out), _stream(stream)))
        return out

    def phi_of(self, f, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(self.lib.lbm_phi_of(self.ctx, _ptr(f), _ptr(out), _stream(stream)))
        return out

    def current(self):
        fp, pp, t = _VP(), _VP(), ctypes.c_longlong()
        _check(self.lib.lbm_current(self.ctx, ctypes.byref(fp), ctypes.byref(pp), ctypes.byref(t)))
        which = 0 if fp.value == self.f[0].data_ptr() else 1
        return which, t.value

    def set_current(self, which, t):
        _check(self.lib.lbm_set_current(self.ctx, int(which), int(t)))

    def set_nontemporal(self, on):
        _check(self.lib.lbm_set_nontemporal(self.ctx, int(bool(on))))

    def set_chunk(self, chunk):
        _check(self.lib.lbm_set_chunk(self.ctx, int(chunk)))

    def set_remap(self, on):
        """XCD-aware workgroup order on or off (lbm_set_remap)."""
        _check(self.lib.lbm_set_remap(self.ctx, int(bool(on))))

    def tune(self, reps=5, stream=None):
        """Autotune the launch shape; restarts from the phi0 given to init."""
        buf = ctypes.create_string_buffer(4096)
        _check(self.lib.lbm_tune(self.ctx, int(reps), _stream(stream), buf, len(buf)))
        return buf.value.decode()

    def set_two_step(self, on, shape=0):
        """Two time steps per pass inside step() (where lbm_set_two_step
        applies), with tile shape `shape` (lbm_set_two_step, two_step_shapes)."""
        _check(self.lib.lbm_set_two_step(self.ctx, 1 + int(shape) if on else 0))

    def two_step_shapes(self):
        """[(rows, waves per workgroup)] of the two-step tile shapes."""
        out, i = [], 0
        r, w = ctypes.c_int(), ctypes.c_int()
        while self.lib.lbm_two_step_shape(self.ctx, i, ctypes.byref(r), ctypes.byref(w)) == 0:
            out.append((r.value, w.value))
            i += 1
        return out

    def set_check(self, every):
        _check(self.lib.lbm_set_check(self.ctx, int(every)))

    def recenter(self, stream=None):
        """Move phi_ref to the mean of phi and shift the stored offsets to match."""
        _check(self.lib.lbm_recenter(self.ctx, _stream(stream)))

    def set_recenter(self, every):
        """Re-centre inside step() every `every` steps (0 = never)."""
        _check(self.lib.lbm_set_recenter(self.ctx, int(every)))

    def set_phi_wall(self, lo, hi, stream=None):
        """New Dirichlet values of the two walls, used by the next gather."""
        _check(self.lib.lbm_set_phi_wall(self.ctx, float(lo), float(hi), _stream(stream)))

    def set_fields(self, k0_field=None, r_field=None):
        """Bind per-node fields (FP64 device tensors, kept alive here): K0(x) as
        [..., 3] (2-D: xx, yy, xy) or [..., 6] (3-D: xx, yy, zz, xy, yz, xz), and
        an external source R(x) (Scheme B), [nz][ny][nx] or [ny][nx].  Rewrite
        the source tensor in place between steps for R(x, t)."""
        import torch
        for t in (k0_field, r_field):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda"):
                raise ValueError("fields must be contiguous float64 CUDA tensors")
        nk = 3 if self.q == 9 else 6
        if k0_field is not None and k0_field.numel() != self.N * nk:
            raise ValueError(f"k0_field needs {nk} values per node")
        if r_field is not None and r_field.numel() != self.N:
            raise ValueError("r_field needs one value per node")
        self._fields = (k0_field, r_field)
        _check(self.lib.lbm_set_fields(self.ctx, _ptr(k0_field), _ptr(r_field)))

    def set_k0(self, k0):
        arr = (ctypes.c_double * 9)(*np.asarray(k0, dtype=np.float64).reshape(-1).tolist())
        _check(self.lib.lbm_set_k0(self.ctx, arr))

    def reduce(self, phi, ref=None, stream=None):
        out = (ctypes.c_double * 8)()
        _check(self.lib.lbm_reduce(self.ctx, _ptr(phi), _ptr(ref), out, _stream(stream)))
        keys = ("sum", "sumsq", "sum_d2", "sum_ref2", "min", "max", "nonfinite", "sum_absd")
        return dict(zip(keys, list(out)))

    def reduce_async(self, phi, ref=None, out=None, stream=None):
        """The reductions of reduce() into a device tensor of 8 FP64 values
        (same order), enqueued on the stream without waiting."""
        import torch
        if out is None:
            out = torch.empty(8, dtype=torch.float64, device=self.device)
        _check(self.lib.lbm_reduce_async(self.ctx, _ptr(phi), _ptr(ref), _ptr(out), _stream(stream)))
        return out

    def reduce_state(self, ref=None, out=None, stream=None):
        """The reductions of reduce() over phi of the current state, formed
        from the populations in one pass (no phi field), into a device tensor
        of 8 FP64 values, enqueued without waiting."""
        import torch
        if out is None:
            out = torch.empty(8, dtype=torch.float64, device=self.device)
        _check(self.lib.lbm_reduce_state(self.ctx, _ptr(ref), _ptr(out), _stream(stream)))
        return out

    # -- adjoint -------------------------------------------------------------
    def adjoint_buffers(self):
        """(psi, pi) buffers of the adjoint variables."""
        import torch
        nb = ctypes.c_size_t()
        _check(self.lib.lbm_adjoint_bytes(self.ctx, ctypes.byref(nb)))
        psi = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        pi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        return psi, pi

    def adjoint_seed(self, gphi, psi, pi, stream=None):
        _check(self.lib.lbm_adjoint_seed(self.ctx, _ptr(gphi), _ptr(psi), _ptr(pi), _stream(stream)))

    def adjoint_step(self, f_s, p_s, psi_next, pi_next, psi_out, pi_out, stream=None):
        _check(self.lib.lbm_adjoint_step(self.ctx, _ptr(f_s), _ptr(p_s), _ptr(psi_next), _ptr(pi_next),
                                         _ptr(psi_out), _ptr(pi_out), _stream(stream)))

    @property
    def adjoint_pair_ok(self):
        """Whether adjoint_step2 (two reversed sweeps per launch) applies."""
        ok = ctypes.c_int()
        _check(self.lib.lbm_adjoint_pair_ok(self.ctx, ctypes.byref(ok)))
        return bool(ok.value)

    def adjoint_tile_shapes(self):
        """[(rows, waves per workgroup)] of the adjoint_step2 tile shapes."""
        out, i = [], 0
        r, w = ctypes.c_int(), ctypes.c_int()
        while self.lib.lbm_adjoint_tile_shape(self.ctx, i, ctypes.byref(r), ctypes.byref(w)) == 0:
            out.append((r.value, w.value))
            i += 1
        return out

    @property
    def adjoint_tile(self):
        """Index of the adjoint_step2 tile shape in use (adjoint_tile_shapes)."""
        s = ctypes.c_int()
        _check(self.lib.lbm_adjoint_tile(self.ctx, ctypes.byref(s)))
        return s.value

    def set_adjoint_tile(self, shape=None):
        """Force adjoint_step2 tile shape `shape`; None restores the pick made
        at creation."""
        _check(self.lib.lbm_set_adjoint_tile(self.ctx, 0 if shape is None else 1 + int(shape)))

    def adjoint_pairs_faster(self, reps=8, trials=3, shapes=True):
        """Whether two reversed sweeps per launch beat two one-sweep launches
        here, and in which tile shape: the one-sweep kernel and the pair in
        every tile shape are timed `trials` times, alternately, on scratch
        buffers (zero adjoint variables, the current forward state).  The
        pair keeps the shape picked at creation unless another is at least 2%
        faster (set_adjoint_tile), and pairs are taken only when their best
        time per sweep is at least 2% below the one-sweep kernel's best, so
        that near-ties resolve the same way in every run (shapes=False: only
        the picked shape is timed).  The answer is kept.  The trial adds to
        the K0 sums, so call it before lbm_adjoint_seed, which clears them."""
        import torch
        if getattr(self, "_adj_pairs", None) is not None:
            return self._adj_pairs
        if not self.adjoint_pair_ok:
            self._adj_pairs = False
            return False
        which, _ = self.current()
        f, p = self.f[which], self.p
        a, pa = self.adjoint_buffers()
        b, pb = self.adjoint_buffers()
        a.zero_(); pa.zero_(); b.zero_(); pb.zero_()
        picked = self.adjoint_tile
        order = [picked] + ([s for s in range(len(self.adjoint_tile_shapes())) if s != picked] if shapes else [])

        def singles():
            for _ in range(reps):
                self.adjoint_step(f, p, a, pa, b, pa)
                self.adjoint_step(f, p, b, pa, a, pa)

        def pairs(shape):
            self.set_adjoint_tile(shape)
            for _ in range(reps):
                self.adjoint_step2(f, p, f, p, a, pa, b, pb)
                self.adjoint_step2(f, p, f, p, b, pb, a, pa)

        singles()
        for s in order:
            pairs(s)
        per_single = float("inf")
        per_pair = {s: float("inf") for s in order}
        for _ in range(trials):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 + 2 * len(order))]
            ev[0].record(); singles(); ev[1].record()
            for i, s in enumerate(order):
                ev[2 + 2 * i].record(); pairs(s); ev[3 + 2 * i].record()
            torch.cuda.synchronize()
            per_single = min(per_single, ev[0].elapsed_time(ev[1]) / (2 * reps))
            for i, s in enumerate(order):
                per_pair[s] = min(per_pair[s], ev[2 + 2 * i].elapsed_time(ev[3 + 2 * i]) / (4 * reps))
        best = picked
        for s in order[1:]:
            if per_pair[s] < 0.98 * per_pair[best]:
                best = s
        self.set_adjoint_tile(best)
        self._adj_pairs = per_pair[best] < 0.98 * per_single
        return self._adj_pairs

    def adjoint_step2(self, f_s, p_s, f_sm1, p_sm1, psi_next, pi_next, psi_out, pi_out, stream=None):
        """Reversed sweeps s and s - 1 in one launch: (psi_{s+1}, pi_{s+1}) ->
        (psi_{s-1}, pi_{s-1}); pi_out must differ from pi_next."""
        _check(self.lib.lbm_adjoint_step2(self.ctx, _ptr(f_s), _ptr(p_s), _ptr(f_sm1), _ptr(p_sm1),
                                          _ptr(psi_next), _ptr(pi_next), _ptr(psi_out), _ptr(pi_out),
                                          _stream(stream)))

    def adjoint_init(self, phi0, psi0, pi0, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(self.lib.lbm_adjoint_init(self.ctx, _ptr(phi0), _ptr(psi0), _ptr(pi0), _ptr(out),
                                         _stream(stream)))
        return out

    def adjoint_grad_k0(self, stream=None):
        out = (ctypes.c_double * 6)()
        _check(self.lib.lbm_adjoint_grad_k0(self.ctx, out, _stream(stream)))
        v = list(out)
        return {"xx": v[0], "xy": v[1], "yy": v[2], "xz": v[3], "yz": v[4], "zz": v[5]}

    # -- views ---------------------------------------------------------------
    def storage_view(self, buf):
        """Typed [q, N] view of a distribution buffer (offsets f - w phi_ref);
        planes are padded apart, so the view is strided."""
        import torch
        dt = {0: torch.float64, 1: torch.float32, 2: torch.float16}[self.desc.precision]
        t = buf.view(dt)
        plane = self.plane_elems()
        return t[: self.q * plane].view(self.q, plane)[:, : self.N]

    def plane_elems(self):
        """Elements between consecutive direction planes."""
        import torch
        dt = {0: torch.float64, 1: torch.float32, 2: torch.float16}[self.desc.precision]
        nb = ctypes.c_size_t()
        _check(self.lib.lbm_adjoint_bytes(self.ctx, ctypes.byref(nb)))
        # psi uses the same plane stride in the compute type
        return nb.value // (8 if self.desc.precision == 0 else 4) // self.q


def reduce_noalloc(phi, ref=None, out=None, n=None, stream=None):
    """The 8 FP64 reductions of Lbm.reduce_async over the first n values of a
    float64 device tensor (default: all), with no context and no allocation
    in the library (lbm_reduce_noalloc); `out` (8 float64 values on the
    device) is allocated here by torch when not given."""
    import torch
    if out is None:
        out = torch.empty(8, dtype=torch.float64, device=phi.device)
    n = phi.numel() if n is None else int(n)
    _check(load().lbm_reduce_noalloc(_ptr(phi), _ptr(ref), ctypes.c_size_t(n), _ptr(out), _stream(stream)))
    return out


def probe_copy(src, dst, grid=0, stream=None):
    """Plain 16-byte-per-lane device copy of src into dst (torch tensors)."""
    n = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    _check(load().lbm_probe_copy(_ptr(src), _ptr(dst), ctypes.c_size_t(n & ~15), int(grid), _stream(stream)))


class Batch:
    """Many independent D2Q9 instances advanced together (lbm_batch_*)."""

    def __init__(self, specs, device="cuda"):
        import torch
        self.lib = load()
        self.specs = list(specs)
        arr = (LbmDesc * len(self.specs))(*[desc_from_spec(sp) for sp in self.specs])
        b = _VP()
        _check(self.lib.lbm_batch_create(arr, len(self.specs), ctypes.byref(b)))
        self.b = b
        fb, pb, tn = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_longlong()
        _check(self.lib.lbm_batch_layout(self.b, ctypes.byref(fb), ctypes.byref(pb), ctypes.byref(tn)))
        self.total_nodes = tn.value
        self.device = torch.device(device)
        self.f = [torch.empty(fb.value, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.p = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        self.offsets, self.shapes = [], []
        for i in range(len(self.specs)):
            off, nx, ny = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int()
            _check(self.lib.lbm_batch_instance(self.b, i, ctypes.byref(off), ctypes.byref(nx), ctypes.byref(ny)))
            self.offsets.append(off.value)
            self.shapes.append((ny.value, nx.value))

    def __del__(self):
        try:
            if getattr(self, "b", None):
                self.lib.lbm_batch_destroy(self.b)
                self.b = None
        except Exception:
            pass

    def pack(self, fields):
        """Concatenate per-instance [ny][nx] fields into one FP64 device arena."""
        import torch
        arena = torch.empty(self.total_nodes, dtype=torch.float64, device=self.device)
        for off, shp, fld in zip(self.offsets, self.shapes, fields):
            n = shp[0] * shp[1]
            arena[off:off + n] = torch.as_tensor(np.ascontiguousarray(fld).reshape(-1), dtype=torch.float64)
        return arena

    def unpack(self, arena):
        return [arena[off:off + s[0] * s[1]].view(s) for off, s in zip(self.offsets, self.shapes)]

    def init(self, phi0_fields, stream=None):
        self._phi0 = self.pack(phi0_fields)
        _check(self.lib.lbm_batch_init(self.b, _ptr(self._phi0), _ptr(self.f[0]), _ptr(self.f[1]), _ptr(self.p),
                                       _stream(stream)))
        return self

    def step(self, n=1, stream=None):
        _check(self.lib.lbm_batch_step(self.b, int(n), _stream(stream)))

    def phi(self, stream=None):
        import torch
        out = torch.empty(self.total_nodes, dtype=torch.float64, device=self.device)
        _check(self.lib.lbm_batch_get_phi(self.b, _ptr(out), _stream(stream)))
        return out

    def tune(self, reps=5, use_cache=False, stream=None):
        buf = ctypes.create_string_buffer(8192)
        _check(self.lib.lbm_batch_tune(self.b, int(reps), int(use_cache), _stream(stream), buf, len(buf)))
        return buf.value.decode()

    def set_shape(self, shape, grid=0, remap=1):
        _check(self.lib.lbm_batch_set_shape(self.b, int(shape), int(grid), int(remap)))

    def get_shape(self):
        s, g, r, wg, npt = (ctypes.c_int(), ctypes.c_uint(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int())
        _check(self.lib.lbm_batch_get_shape(self.b, ctypes.byref(s), ctypes.byref(g), ctypes.byref(r),
                                            ctypes.byref(wg), ctypes.byref(npt)))
        return {"shape": s.value, "grid": g.value, "remap": r.value, "wg": wg.value, "npt": npt.value}
