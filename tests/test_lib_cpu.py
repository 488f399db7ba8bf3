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
    assert G._lib.gmg_residual_noalloc(None, 0, 0, None, None, None, None, None) == G.GMG_EINVAL
    assert G._lib.gmg_destroy(None) == G.GMG_OK


def test_copy_probe_validation():
    import paper_1402_3545_amd as G
    lib = G._lib
    assert lib.gmg_copy_probe(None, None, 8, None) == -1
    assert lib.gmg_copy_probe(C.c_void_p(0x1000), C.c_void_p(0x2000), 12, None) == -1  # not 8k
    assert lib.gmg_copy_probe(C.c_void_p(0x1000), C.c_void_p(0x2000), -8, None) == -1
    assert lib.gmg_copy_probe(C.c_void_p(0x1008), C.c_void_p(0x2000), 8, None) == -1  # align
    assert lib.gmg_copy_probe(C.c_void_p(0x1000), C.c_void_p(0x1010), 64, None) == -1  # overlap


class _StubCtx:
    """Stands in for a context on a machine without a GPU: the binding checks
    every field against the layout before any call reaches the library."""
    nlevels, prec_precond, rho, device, handle = 2, 0, 2.0 / 3.0, None, None

    def layout(self, level=0):
        return (32, 16 * 8 * 32) if level == 0 else (32, 8 * 8 * 32)

    def shape(self, level=0):
        return 16 >> level, 16 >> level, 8


def _misuse_cases():
    import torch
    n0, n1 = 16 * 8 * 32, 8 * 8 * 32
    ok = torch.zeros(n0, dtype=torch.float64)
    return [
        ("float32 f in an FP64 solve", "gmg_solve",
         (torch.zeros(n0, dtype=torch.float32), ok)),
        ("integer field", "spmv", (0, torch.zeros(n0, dtype=torch.int64), ok)),
        ("mixed precisions", "spmv", (0, ok, torch.zeros(n0, dtype=torch.float32))),
        ("unpadded nx*ny*nz field", "gmg_solve", (torch.zeros(16 * 16 * 8), ok)),
        ("non-contiguous field", "line_solve",
         (0, torch.zeros(2 * n0, dtype=torch.float64)[::2], ok)),
        ("coarse field on the fine level", "line_smooth",
         (0, torch.zeros(n1, dtype=torch.float64), ok)),
        ("level out of range", "spmv", (2, ok, ok)),
        ("restriction onto level 0", "gmg_restrict_smooth", (0, ok, ok, ok)),
        ("vcycle field in the wrong precision", "gmg_vcycle",
         (torch.zeros(n0, dtype=torch.float32), torch.zeros(n0, dtype=torch.float32))),
        ("host tensor", "gmg_residual", (0, ok, ok, ok)),
        ("not a tensor", "pcg_solve", (None, ok)),
    ]


@pytest.mark.parametrize("case", range(11))
def test_binding_rejects_misfit_fields_before_any_launch(case):
    """The C ABI takes no lengths, so the binding checks type, precision,
    contiguity, the padded element count and the device of every field first;
    each misuse raises ValueError (the stub context has no library handle, so
    reaching the library would fail differently)."""
    import paper_1402_3545_amd as G
    what, fn, args = _misuse_cases()[case]
    with pytest.raises(ValueError):
        getattr(G, fn)(_StubCtx(), *args)


def test_binding_rejects_misfit_batched_fields():
    import torch
    import paper_1402_3545_amd as G

    class _StubBatch:
        ninst, nrhs, device, handle = 1, 2, None, None

        def layout(self, instance):
            return 32, 512

    ok = torch.zeros(512, dtype=torch.float64)
    with pytest.raises(ValueError):
        G.gmg_batch_solve(_StubBatch(), [ok, torch.zeros(100, dtype=torch.float64)], [ok, ok])
    with pytest.raises(ValueError):
        G.gmg_batch_solve(_StubBatch(), [ok, ok], [ok, ok.float()])
    with pytest.raises(ValueError):  # host tensors
        G.gmg_batch_solve(_StubBatch(), [ok, ok], [ok, ok])
