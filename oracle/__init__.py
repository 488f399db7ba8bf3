"""ctypes wrapper of the plain FP64 CPU oracle.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package.  It loads oracle/liboracle.so (built by
oracle/build.py from oracle.c with gcc) and shares no code with the HIP library.

Vectors are numpy float64 arrays in the canonical order (j*nx + i)*nz + k.
Levels are numbered by depth (0 = finest).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = C.CDLL(_build.LIB)
    lib.or_create.restype = C.c_void_p
    lib.or_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                              C.c_double, _D, _D, C.c_double, C.c_int]
    lib.or_create_matfree.restype = C.c_void_p
    lib.or_create_matfree.argtypes = lib.or_create.argtypes
    lib.or_apply_rows.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.POINTER(C.c_int64), _D, _D]
    lib.or_residual_norm2_rows.restype = C.c_double
    lib.or_residual_norm2_rows.argtypes = [C.c_void_p, C.c_int, _D, _D]
    lib.or_line_solve_columns.argtypes = [C.c_void_p, C.c_int, C.c_int64,
                                          C.POINTER(C.c_int64), _D, _D]
    lib.or_destroy.argtypes = [C.c_void_p]
    lib.or_last_error.restype = C.c_char_p
    lib.or_shape.argtypes = [C.c_void_p, C.c_int, _I, _I, _I]
    lib.or_nnz.restype = C.c_int64
    lib.or_nnz.argtypes = [C.c_void_p, C.c_int]
    lib.or_csr.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32), _D]
    lib.or_profiles.argtypes = [C.c_void_p, _D, _D]
    lib.or_faces.argtypes = [C.c_void_p, C.c_int, _D, _D, _D]
    lib.or_walls.argtypes = [C.c_void_p, C.c_int, _D]
    for name in ("or_spmv", "or_line_solve"):
        getattr(lib, name).argtypes = [C.c_void_p, C.c_int, _D, _D]
    lib.or_residual.argtypes = [C.c_void_p, C.c_int, _D, _D, _D]
    lib.or_smooth.argtypes = [C.c_void_p, C.c_int, _D, _D, C.c_double]
    lib.or_restrict.argtypes = [C.c_void_p, C.c_int, _D, _D]
    lib.or_prolongate_add.argtypes = [C.c_void_p, C.c_int, _D, _D]
    lib.or_restrict_smooth.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, C.c_double]
    lib.or_vcycle.argtypes = [C.c_void_p, _D, _D]
    lib.or_mg_solve.argtypes = [C.c_void_p, _D, _D, C.c_double, C.c_int, _I, _D]
    lib.or_pcg_solve.argtypes = [C.c_void_p, _D, _D, C.c_double, C.c_int, _I, _D, _D]
    lib.or_dot.restype = C.c_double
    lib.or_dot.argtypes = [C.c_int64, _D, _D]
    lib.or_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def num_threads() -> int:
    return _load().or_num_threads()


class OracleProblem:
    """The discrete operator hierarchy, assembled as CSR on the host."""

    def __init__(self, nx, ny, nz, nlevels=1, kv=1.0, sigma=1.0, zfaces=None, kh=None,
                 bc_v=0, rho=2.0 / 3.0, ncoarse=2, matfree=False, bc_h=0):
        lib = _load()
        self.nx, self.ny, self.nz, self.nlevels = int(nx), int(ny), int(nz), int(nlevels)
        self.rho = float(rho)
        self.bc_h, self.bc_v = int(bc_h), int(bc_v)
        zf = None if zfaces is None else np.ascontiguousarray(zfaces, dtype=np.float64)
        kk = None if kh is None else np.ascontiguousarray(kh, dtype=np.float64)
        if zf is not None and zf.size != nz + 1:
            raise ValueError("zfaces needs nz+1 entries")
        if kk is not None and kk.size != nx * ny:
            raise ValueError("kh needs nx*ny entries")
        create = lib.or_create_matfree if matfree else lib.or_create
        h = create(nx, ny, nz, nlevels, int(bc_h), bc_v, float(kv), float(sigma),
                          _p(zf) if zf is not None else None,
                          _p(kk) if kk is not None else None, float(rho), int(ncoarse))
        if not h:
            raise ValueError(lib.or_last_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    def _chk(self, rc):
        if rc < 0:
            raise RuntimeError(_lib.or_last_error().decode())
        return rc

    def shape(self, depth=0):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._chk(_lib.or_shape(self._h, depth, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def size(self, depth=0):
        nx, ny, nz = self.shape(depth)
        return nx * ny * nz

    def csr(self, depth=0):
        n = self.size(depth)
        nnz = _lib.or_nnz(self._h, depth)
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz, dtype=np.float64)
        self._chk(_lib.or_csr(self._h, depth, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                              col.ctypes.data_as(C.POINTER(C.c_int32)), _p(val)))
        return rp, col, val

    def scipy(self, depth=0):
        import scipy.sparse as sp
        rp, col, val = self.csr(depth)
        n = self.size(depth)
        return sp.csr_matrix((val, col, rp), shape=(n, n))

    def profiles(self):
        dz = np.zeros(self.nz)
        tf = np.zeros(self.nz + 1)
        _lib.or_profiles(self._h, _p(dz), _p(tf))
        return dz, tf

    def faces(self, depth=0):
        nx, ny, _ = self.shape(depth)
        kc, cx, cy = (np.zeros(nx * ny) for _ in range(3))
        self._chk(_lib.or_faces(self._h, depth, _p(kc), _p(cx), _p(cy)))
        return kc, cx, cy

    def walls(self, depth=0):
        nx, ny, _ = self.shape(depth)
        w = np.zeros(nx * ny)
        self._chk(_lib.or_walls(self._h, depth, _p(w)))
        return w

    def _vec(self, x, depth):
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.size != self.size(depth):
            raise ValueError("vector size does not match level")
        return x

    def spmv(self, x, depth=0):
        x = self._vec(x, depth)
        y = np.empty_like(x)
        self._chk(_lib.or_spmv(self._h, depth, _p(x), _p(y)))
        return y

    def residual(self, f, u, depth=0):
        f, u = self._vec(f, depth), self._vec(u, depth)
        r = np.empty_like(f)
        self._chk(_lib.or_residual(self._h, depth, _p(f), _p(u), _p(r)))
        return r

    def line_solve(self, r, depth=0):
        r = self._vec(r, depth)
        z = np.empty_like(r)
        self._chk(_lib.or_line_solve(self._h, depth, _p(r), _p(z)))
        return z

    def smooth(self, f, u, rho=None, depth=0):
        f = self._vec(f, depth)
        u = self._vec(u, depth).copy()
        self._chk(_lib.or_smooth(self._h, depth, _p(f), _p(u),
                                 self.rho if rho is None else float(rho)))
        return u

    def restrict(self, rf, depth_fine=0):
        rf = self._vec(rf, depth_fine)
        fc = np.empty(self.size(depth_fine + 1))
        self._chk(_lib.or_restrict(self._h, depth_fine, _p(rf), _p(fc)))
        return fc

    def prolongate_add(self, uc, uf, depth_coarse=1):
        uc = self._vec(uc, depth_coarse)
        uf = self._vec(uf, depth_coarse - 1).copy()
        self._chk(_lib.or_prolongate_add(self._h, depth_coarse, _p(uc), _p(uf)))
        return uf

    def restrict_smooth(self, rf, depth_coarse=1, rho=None):
        rf = self._vec(rf, depth_coarse - 1)
        n = self.size(depth_coarse)
        fc, uc = np.empty(n), np.empty(n)
        self._chk(_lib.or_restrict_smooth(self._h, depth_coarse, _p(rf), _p(fc), _p(uc),
                                          self.rho if rho is None else float(rho)))
        return fc, uc

    def vcycle(self, f, u):
        f = self._vec(f, 0)
        u = self._vec(u, 0).copy()
        self._chk(_lib.or_vcycle(self._h, _p(f), _p(u)))
        return u

    def mg_solve(self, f, u0=None, rtol=1e-8, maxit=100):
        f = self._vec(f, 0)
        u = np.zeros_like(f) if u0 is None else self._vec(u0, 0).copy()
        it = C.c_int()
        hist = np.zeros(maxit + 1)
        st = self._chk(_lib.or_mg_solve(self._h, _p(f), _p(u), float(rtol), int(maxit),
                                        C.byref(it), _p(hist)))
        return u, it.value, hist[: it.value + 1].copy(), st

    def pcg_solve(self, f, u0=None, rtol=1e-8, maxit=1000):
        f = self._vec(f, 0)
        u = np.zeros_like(f) if u0 is None else self._vec(u0, 0).copy()
        it = C.c_int()
        hist = np.zeros(maxit + 1)
        rt = C.c_double()
        st = self._chk(_lib.or_pcg_solve(self._h, _p(f), _p(u), float(rtol), int(maxit),
                                         C.byref(it), _p(hist), C.byref(rt)))
        return u, it.value, hist[: it.value + 1].copy(), rt.value, st

    # -- row-wise forms (also available without the CSR matrices) ------------
    def apply_rows(self, rows, x, depth=0):
        """(A x) at the given canonical row indices."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        x = self._vec(x, depth)
        y = np.empty(rows.size)
        self._chk(_lib.or_apply_rows(self._h, depth, rows.size,
                                     rows.ctypes.data_as(C.POINTER(C.c_int64)), _p(x), _p(y)))
        return y

    def residual_norm2_rows(self, f, u, depth=0):
        f, u = self._vec(f, depth), self._vec(u, depth)
        v = _lib.or_residual_norm2_rows(self._h, depth, _p(f), _p(u))
        if v < 0:
            raise RuntimeError(_lib.or_last_error().decode())
        return v

    def line_solve_columns(self, cols, r, depth=0):
        """M^{-1} r on the listed columns (index j*nx+i); other entries are NaN."""
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        r = self._vec(r, depth)
        z = np.full_like(r, np.nan)
        self._chk(_lib.or_line_solve_columns(self._h, depth, cols.size,
                                             cols.ctypes.data_as(C.POINTER(C.c_int64)), _p(r),
                                             _p(z)))
        return z

    def column_rows(self, cols, depth=0):
        """Canonical row indices of all layers of the listed columns."""
        nz = self.nz
        cols = np.asarray(cols, dtype=np.int64)
        return (cols[:, None] * nz + np.arange(nz)[None, :]).reshape(-1)
