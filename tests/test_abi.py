"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/lbm.h declares, and rejects invalid descriptions before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1603_09577_amd import lbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1603_09577_amd import build
        build.build()
    return lbm.load()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(lbm_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_exported(L):
    names = declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbm.EXPORTS) == names


def test_descriptor_layout_matches_header():
    """The ctypes mirror has the C struct's size (doubles and ints, natural alignment)."""
    # 4 ints, 3 bc, 6 phi_wall, precision, phi_ref, scheme, d, 19 s, 27 b, 9 dpoly,
    # 9 dten, 9 k0, 9 kpoly, 9 rpoly, flags
    size = ctypes.sizeof(lbm.LbmDesc)
    assert size % 8 == 0 and size > 8 * (6 + 19 + 27 + 9 * 5)


def _create(L, spec, **over):
    d = lbm.desc_from_spec(spec)
    for k, v in over.items():
        setattr(d, k, v)
    ctx = ctypes.c_void_p()
    rc = L.lbm_create(ctypes.byref(d), ctypes.byref(ctx))
    return rc, L.lbm_last_error().decode()


@pytest.mark.parametrize("field,value", [
    ("lattice", 15), ("nx", 0), ("ny", -3), ("d", 0.0), ("d", -1.0), ("precision", 7), ("scheme", 4),
])
def test_invalid_descriptions(L, field, value):
    rc, msg = _create(L, W.spec_nonlinear_2d(16), **{field: value})
    assert rc == lbm.LBM_E_INVALID, msg


def test_invalid_rates_and_tensors(L):
    spec = W.spec_nonlinear_2d(16)
    for bad in (0.0, 2.0, -0.5, 2.5):
        sp = dict(spec)
        sp["s"] = list(spec["s"])
        sp["s"][4] = bad
        rc, msg = _create(L, sp)
        assert rc == lbm.LBM_E_INVALID and "rates" in msg
    sp = dict(spec)
    sp["k0"] = [[0.01, 0.02, 0], [0.02, 0.01, 0], [0, 0, 0]]      # indefinite
    assert _create(L, sp)[0] == lbm.LBM_E_INVALID
    sp["k0"] = [[0.01, 0.002, 0], [0.001, 0.01, 0], [0, 0, 0]]    # not symmetric
    assert _create(L, sp)[0] == lbm.LBM_E_INVALID
    sp = dict(spec)
    sp["kpoly"] = [0.0, 1.0]
    assert _create(L, sp)[0] == lbm.LBM_E_INVALID
    sp = dict(spec)
    sp["dten"] = [[1, 0.1, 0], [0.2, 1, 0], [0, 0, 1]]
    assert _create(L, sp)[0] == lbm.LBM_E_INVALID


def test_unsupported_combinations(L):
    spec = W.spec_nonlinear_2d(16)
    sp = dict(spec)
    sp["bc"] = ["abb", "periodic", "periodic"]
    assert _create(L, sp)[0] == lbm.LBM_E_UNSUPPORTED
    sp = dict(spec)
    sp["scheme"] = "B"
    sp["rpoly"] = [0.0, 0.1, 0.0, -0.1]
    assert _create(L, sp)[0] == lbm.LBM_E_UNSUPPORTED        # Scheme B: Eq. 35 in closed form up to degree 2
    for rp in ([], [1e-3], [0.0, 0.1, -0.1]):                   # no source, constant, quadratic R(phi)
        sp["rpoly"] = rp
        rc, msg = _create(L, sp)
        assert rc in (lbm.LBM_OK, lbm.LBM_E_HIP), msg           # valid; needs a GPU
    sp = W.spec_d3q19_aniso((8, 8, 8), K=np.diag([0.01, 0.02, 0.03]))
    sp["bc"] = ["periodic", "abb", "periodic"]
    assert _create(L, sp)[0] == lbm.LBM_E_UNSUPPORTED


def test_too_many_nodes(L):
    spec = W.spec_d3q19_aniso((1 << 11, 1 << 10, 1 << 10), K=np.diag([0.01, 0.02, 0.03]))
    assert _create(L, spec)[0] == lbm.LBM_E_INVALID


def test_null_arguments(L):
    ctx = ctypes.c_void_p()
    assert L.lbm_create(None, ctypes.byref(ctx)) == lbm.LBM_E_INVALID
    assert L.lbm_step(None, 1, None) == lbm.LBM_E_INVALID
    assert L.lbm_get_phi(None, None, None) == lbm.LBM_E_INVALID
    assert L.lbm_adjoint_step(None, None, None, None, None, None, None, None) == lbm.LBM_E_INVALID
    assert L.lbm_adjoint_step2(*([None] * 10)) == lbm.LBM_E_INVALID
    assert L.lbm_adjoint_pair_ok(None, None) == lbm.LBM_E_INVALID
    assert L.lbm_adjoint_tile_shape(None, 0, None, None) == lbm.LBM_E_INVALID
    assert L.lbm_set_adjoint_tile(None, 1) == lbm.LBM_E_INVALID
    assert L.lbm_adjoint_tile(None, None) == lbm.LBM_E_INVALID
    assert L.lbm_two_step_shape(None, 0, None, None) == lbm.LBM_E_INVALID
    assert L.lbm_set_remap(None, 1) == lbm.LBM_E_INVALID
    assert L.lbm_recenter(None, None) == lbm.LBM_E_INVALID
    assert L.lbm_set_recenter(None, 5) == lbm.LBM_E_INVALID
    assert L.lbm_set_check(None, 5) == lbm.LBM_E_INVALID
    assert L.lbm_tune(None, 1, None, None, 0) == lbm.LBM_E_INVALID
    assert L.lbm_batch_step(None, 1, None) == lbm.LBM_E_INVALID


def test_rational_flux_needs_remark3(L):
    spec = W.spec_nonlinear_2d(16)
    spec["bden"] = [1.0, -2.0, 2.0]
    rc, msg = _create(L, spec)
    assert rc == lbm.LBM_E_UNSUPPORTED and "REMARK3" in msg
    spec["flags"] = lbm.FLAG_REMARK3
    rc, msg = _create(L, spec)
    assert rc in (lbm.LBM_OK, lbm.LBM_E_HIP), msg
    spec["bden"] = [1.0, float("nan")]
    assert _create(L, spec)[0] == lbm.LBM_E_INVALID
