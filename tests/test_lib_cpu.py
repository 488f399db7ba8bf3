"""CPU-side checks of the HIP library: it loads, exports every entry point that
include/gmg.h declares, and rejects invalid parameters before touching the GPU
(validation runs before any HIP call)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|const char\s*\*|char\s*\*)\s*\**\s*(\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("gmg_setup", "gmg_vcycle", "pcg_solve", "spmv", "line_smooth"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1402_3545_amd as G
    lib = C.CDLL(G.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(G.EXPORTS) <= set(_declared())


def _params(**kw):
    import paper_1402_3545_amd as G
    p = G.GmgParams()
    G._lib.gmg_default_params(C.byref(p))
    p.nx, p.ny, p.nz, p.nlevels = 16, 16, 8, 2
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,status", [
    ({"nz": 1}, -1), ({"nz": 200}, -5), ({"nx": 6, "nlevels": 3}, -1),
    ({"nx": 4, "nlevels": 4}, -1), ({"bc_h": 2}, -1), ({"bc_h": -1}, -1), ({"bc_v": 2}, -1),
    ({"sigma": 0.0}, -1), ({"kv": -1.0}, -1), ({"rho": 0.0}, -1), ({"ncoarse": 0}, -1),
    ({"prec_precond": 3}, -1), ({"nlevels": 0}, -1)])
def test_setup_rejects_invalid_parameters(kw, status):
    import paper_1402_3545_amd as G
    p = _params(**kw)
    h = C.c_void_p()
    st = G._lib.gmg_setup(C.byref(p), None, C.byref(h))
    assert st == status
    assert not h.value
    assert G.gmg_last_error()


def test_setup_rejects_bad_host_arrays():
    import numpy as np
    import paper_1402_3545_amd as G
    kh = -np.ones(256)
    p = _params(kh=kh.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    assert G._lib.gmg_setup(C.byref(p), None, C.byref(h)) == G.GMG_EINVAL
    zf = np.zeros(9)
    p = _params(zfaces=zf.ctypes.data_as(C.POINTER(C.c_double)))
    assert G._lib.gmg_setup(C.byref(p), None, C.byref(h)) == G.GMG_EINVAL
    assert G._lib.gmg_setup(None, None, C.byref(h)) == G.GMG_EINVAL


def test_null_context_is_rejected():
    import paper_1402_3545_amd as G
    assert G._lib.spmv(None, 0, 0, None, None, None) == G.GMG_EINVAL
    assert G._lib.gmg_vcycle(None, None, None, None) == G.GMG_EINVAL
    assert G._lib.gmg_set_launch(None, 0, 0, 0, 4, 0) == G.GMG_EINVAL
    assert G._lib.gmg_get_launch(None, 0, 0, 0, None, None) == G.GMG_EINVAL
    assert G._lib.gmg_autotune(None, 3, None) == G.GMG_EINVAL
    assert G._lib.gmg_timing_filter(None, 1) == G.GMG_EINVAL
    assert G._lib.gmg_destroy(None) == G.GMG_OK


def test_copy_probe_validation():
    import paper_1402_3545_amd as G
    lib = G._lib
    assert lib.gmg_copy_probe(None, None, 8, None) == -1
    assert lib.gmg_copy_probe(C.c_void_p(0x1000), C.c_void_p(0x2000), 12, None) == -1  # not 8k
    assert lib.gmg_copy_probe(C.c_void_p(0x1000), C.c_void_p(0x2000), -8, None) == -1
    assert lib.gmg_copy_probe(C.c_void_p(0x1008), C.c_void_p(0x2000), 8, None) == -1  # align
    assert lib.gmg_copy_probe(C.c_void_p(0x1000), C.c_void_p(0x1010), 64, None) == -1  # overlap
