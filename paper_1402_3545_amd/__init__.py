"""Python binding of libgmg.so, the gfx950 tensor-product multigrid / line-CG library.

Argument marshalling only: every step of the solvers runs in the HIP kernels
behind the C ABI declared in include/gmg.h.  The functions keep the C names
(gmg_setup, spmv, line_solve, line_smooth, gmg_residual, gmg_restrict_smooth,
gmg_prolongate, gmg_vcycle, gmg_solve, pcg_solve, ...); fields are torch CUDA
tensors in the library layout and the current torch stream is passed down.

There is no fallback: importing the package raises if the library is missing.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

LIB_PATH = _build.LIB

GMG_OK, GMG_EINVAL, GMG_ENOMEM, GMG_EHIP, GMG_ENOCONV, GMG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GMG_F64, GMG_F32 = 0, 1

EXPORTS = ("gmg_default_params", "gmg_setup", "gmg_destroy", "gmg_field_layout", "spmv",
           "line_solve", "line_smooth", "gmg_residual", "gmg_residual_noalloc",
           "gmg_restrict_smooth", "gmg_prolongate",
           "gmg_vcycle", "gmg_solve", "pcg_solve", "gmg_batch_setup", "gmg_batch_layout",
           "gmg_batch_solve", "gmg_timing_enable", "gmg_timing_read", "gmg_timing_filter",
           "gmg_set_launch",
           "gmg_get_launch", "gmg_autotune", "gmg_set_graphs", "gmg_solver_polls",
           "gmg_transpose_in",
           "gmg_transpose_out",
           "gmg_solve_host", "gmg_copy_probe", "gmg_last_error")

# kernel ids of the timing facility (gmg_kernel in include/gmg.h)
KERNELS = ("spmv", "residual", "line_solve", "smooth", "restrict_smooth", "prolongate",
           "cg_spmv", "cg_tridiag", "reduce", "aux", "correct", "fcg",
           "residual_restrict", "prolong_smooth")


class GmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"status {status}: {message}")
        self.status = status


class GmgParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nlevels", C.c_int32),
                ("bc_h", C.c_int32), ("bc_v", C.c_int32), ("kv", C.c_double),
                ("sigma", C.c_double), ("zfaces", C.POINTER(C.c_double)),
                ("kh", C.POINTER(C.c_double)), ("rho", C.c_double), ("ncoarse", C.c_int32),
                ("prec_precond", C.c_int32)]


def canonical_to_xcontig(a, nx, ny, nz, ldx):
    """(j*nx+i)*nz+k host order -> the library layout (j*nz+k)*ldx+i, padding zeroed."""
    a = np.asarray(a)
    v = a.reshape(ny, nx, nz).transpose(0, 2, 1)
    out = np.zeros((ny, nz, ldx), dtype=a.dtype)
    out[:, :, :nx] = v
    return out.reshape(-1)


def xcontig_to_canonical(a, nx, ny, nz, ldx):
    v = np.asarray(a).reshape(ny, nz, ldx)[:, :, :nx]
    return np.ascontiguousarray(v.transpose(0, 2, 1)).reshape(-1)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1402_3545_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64p, dbl, dblp = C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.c_double, \
        C.POINTER(C.c_double)
    intp = C.POINTER(C.c_int)
    sig = {
        "gmg_default_params": (None, [C.POINTER(GmgParams)]),
        "gmg_setup": (i32, [C.POINTER(GmgParams), vp, C.POINTER(vp)]),
        "gmg_destroy": (i32, [vp]),
        "gmg_field_layout": (i32, [vp, i32, i64p, i64p]),
        "spmv": (i32, [vp, i32, i32, vp, vp, vp]),
        "line_solve": (i32, [vp, i32, i32, vp, vp, vp]),
        "line_smooth": (i32, [vp, i32, i32, vp, vp, i32, dbl, vp]),
        "gmg_residual": (i32, [vp, i32, i32, vp, vp, vp, dblp, vp]),
        "gmg_residual_noalloc": (i32, [vp, i32, i32, vp, vp, vp, vp, vp]),
        "gmg_restrict_smooth": (i32, [vp, i32, i32, vp, vp, vp, dbl, vp]),
        "gmg_prolongate": (i32, [vp, i32, i32, vp, vp, vp]),
        "gmg_vcycle": (i32, [vp, vp, vp, vp]),
        "gmg_solve": (i32, [vp, vp, vp, dbl, i32, intp, dblp, dblp, vp]),
        "pcg_solve": (i32, [vp, vp, vp, dbl, i32, i32, intp, dblp, dblp, vp]),
        "gmg_batch_setup": (i32, [C.POINTER(GmgParams), i32, i32, vp, C.POINTER(vp)]),
        "gmg_batch_layout": (i32, [vp, i32, i64p, i64p]),
        "gmg_batch_solve": (i32, [vp, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), dbl, i32, intp,
                                  dblp, vp]),
        "gmg_timing_enable": (i32, [vp, i32]),
        "gmg_timing_read": (i32, [vp, i32, i32, i32, i64p, dblp]),
        "gmg_timing_filter": (i32, [vp, C.c_uint32]),
        "gmg_set_launch": (i32, [vp, i32, i32, i32, i32, i32]),
        "gmg_get_launch": (i32, [vp, i32, i32, i32, intp, intp]),
        "gmg_autotune": (i32, [vp, i32, vp]),
        "gmg_set_graphs": (i32, [vp, i32]),
        "gmg_solver_polls": (i32, [vp]),
        "gmg_transpose_in": (i32, [vp, i32, i32, vp, vp, vp]),
        "gmg_copy_probe": (i32, [vp, vp, C.c_int64, vp]),
        "gmg_transpose_out": (i32, [vp, i32, i32, vp, vp, vp]),
        "gmg_solve_host": (i32, [vp, i32, vp, vp, dbl, i32, intp, dblp, dblp, vp]),
        "gmg_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _check(status: int) -> int:
    if status < 0:
        raise GmgError(status, _lib.gmg_last_error().decode())
    return status


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


_DTYPE_NAME = {GMG_F64: "float64", GMG_F32: "float32"}


def _field(ctx, t, name, level=0, prec=None, elems=None):
    """Check one caller field before its pointer goes to the C ABI, which takes
    no lengths: a torch tensor on the context's GPU, contiguous, of the expected
    element type (prec; None = float64 or float32), holding at least the level's
    padded element count (gmg_field_layout; or `elems`).  Raises ValueError, so
    a misfit never reaches a kernel.  Returns the precision code."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype == torch.float64:
        got = GMG_F64
    elif t.dtype == torch.float32:
        got = GMG_F32
    else:
        raise ValueError(f"{name}: must be float64 or float32, got {t.dtype}")
    if prec is not None and got != prec:
        raise ValueError(f"{name}: must be {_DTYPE_NAME[prec]}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    need = ctx.layout(level)[1] if elems is None else int(elems)
    if t.numel() < need:
        raise ValueError(f"{name}: holds {t.numel()} elements, level {level} needs {need} "
                         "(the padded layout of gmg_field_layout)")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor (device {t.device})")
    dev = getattr(ctx, "device", None)
    if dev is not None and t.device.index != dev:
        raise ValueError(f"{name}: on cuda:{t.device.index}, the context lives on cuda:{dev}")
    return got


def _fields(ctx, spec, prec=None):
    """_field over (tensor, name, level) triples that must share one precision."""
    for t, name, level in spec:
        prec = _field(ctx, t, name, level, prec)
    return prec


def _distinct(a, b, what):
    if a.data_ptr() == b.data_ptr():
        raise ValueError(f"{what} must not be the same buffer")


class GmgContext:
    """Owns a gmg_ctx: the level hierarchy for one operator on the current device."""

    def __init__(self, nx, ny, nz, nlevels=1, kv=1.0, sigma=1.0, zfaces=None, kh=None, bc_v=0,
                 rho=2.0 / 3.0, ncoarse=2, prec_precond=GMG_F64, bc_h=0, stream=None):
        p = GmgParams()
        _lib.gmg_default_params(C.byref(p))
        p.nx, p.ny, p.nz, p.nlevels = int(nx), int(ny), int(nz), int(nlevels)
        p.bc_h, p.bc_v = int(bc_h), int(bc_v)
        p.kv, p.sigma, p.rho, p.ncoarse = float(kv), float(sigma), float(rho), int(ncoarse)
        p.prec_precond = int(prec_precond)
        keep = []
        if zfaces is not None:
            z = np.ascontiguousarray(zfaces, dtype=np.float64)
            if z.size != nz + 1:
                raise ValueError("zfaces needs nz+1 entries")
            keep.append(z)
            p.zfaces = z.ctypes.data_as(C.POINTER(C.c_double))
        if kh is not None:
            k = np.ascontiguousarray(kh, dtype=np.float64)
            if k.size != nx * ny:
                raise ValueError("kh needs nx*ny entries")
            keep.append(k)
            p.kh = k.ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        import torch
        self.device = torch.cuda.current_device() if torch.cuda.is_available() else None
        _check(_lib.gmg_setup(C.byref(p), _stream(stream), C.byref(h)))
        self._h = h
        self.nx, self.ny, self.nz, self.nlevels = p.nx, p.ny, p.nz, p.nlevels
        self.prec_precond = p.prec_precond
        self.rho = p.rho

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gmg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, level=0):
        return self.nx >> level, self.ny >> level, self.nz

    def layout(self, level=0):
        ldx, elems = C.c_int64(), C.c_int64()
        _check(_lib.gmg_field_layout(self._h, int(level), C.byref(ldx), C.byref(elems)))
        return ldx.value, elems.value

    # -- host <-> device layout (plain data movement) -------------------------
    def empty(self, level=0, dtype=None):
        import torch
        dtype = dtype or torch.float64
        _, elems = self.layout(level)
        return torch.zeros(elems, dtype=dtype, device="cuda")

    def to_device(self, canonical, level=0, dtype=None):
        import torch
        nx, ny, nz = self.shape(level)
        ldx, _ = self.layout(level)
        a = canonical_to_xcontig(np.asarray(canonical, dtype=np.float64), nx, ny, nz, ldx)
        t = torch.from_numpy(a)
        if dtype is not None:
            t = t.to(dtype)
        return t.cuda()

    def from_device(self, t, level=0):
        nx, ny, nz = self.shape(level)
        ldx, _ = self.layout(level)
        return xcontig_to_canonical(t.detach().cpu().double().numpy(), nx, ny, nz, ldx)


def _params(nx, ny, nz, nlevels=1, kv=1.0, sigma=1.0, zfaces=None, kh=None, bc_v=0,
            rho=2.0 / 3.0, ncoarse=2, prec_precond=GMG_F64, bc_h=0, keep=None):
    p = GmgParams()
    _lib.gmg_default_params(C.byref(p))
    p.nx, p.ny, p.nz, p.nlevels = int(nx), int(ny), int(nz), int(nlevels)
    p.bc_h, p.bc_v = int(bc_h), int(bc_v)
    p.kv, p.sigma, p.rho, p.ncoarse = float(kv), float(sigma), float(rho), int(ncoarse)
    p.prec_precond = int(prec_precond)
    if zfaces is not None:
        z = np.ascontiguousarray(zfaces, dtype=np.float64)
        if z.size != nz + 1:
            raise ValueError("zfaces needs nz+1 entries")
        keep.append(z)
        p.zfaces = z.ctypes.data_as(C.POINTER(C.c_double))
    if kh is not None:
        k = np.ascontiguousarray(kh, dtype=np.float64)
        if k.size != nx * ny:
            raise ValueError("kh needs nx*ny entries")
        keep.append(k)
        p.kh = k.ctypes.data_as(C.POINTER(C.c_double))
    return p


class GmgBatch:
    """A batched context: independent instances (dicts of GmgContext keyword
    arguments), each with nrhs right-hand sides, solved together."""

    def __init__(self, instances, nrhs=1, stream=None):
        keep = []
        arr = (GmgParams * len(instances))()
        for q, kw in enumerate(instances):
            arr[q] = _params(keep=keep, **kw)
        h = C.c_void_p()
        import torch
        self.device = torch.cuda.current_device() if torch.cuda.is_available() else None
        _check(_lib.gmg_batch_setup(arr, len(instances), int(nrhs), _stream(stream),
                                    C.byref(h)))
        self._h = h
        self.ninst, self.nrhs = len(instances), int(nrhs)
        self.shapes = [(kw["nx"], kw["ny"], kw["nz"]) for kw in instances]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gmg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self, instance):
        ldx, elems = C.c_int64(), C.c_int64()
        _check(_lib.gmg_batch_layout(self._h, int(instance), C.byref(ldx), C.byref(elems)))
        return ldx.value, elems.value

    def to_device(self, canonical, instance):
        import torch
        nx, ny, nz = self.shapes[instance]
        ldx, _ = self.layout(instance)
        return torch.from_numpy(canonical_to_xcontig(np.asarray(canonical, dtype=np.float64),
                                                     nx, ny, nz, ldx)).cuda()

    def from_device(self, t, instance):
        nx, ny, nz = self.shapes[instance]
        ldx, _ = self.layout(instance)
        return xcontig_to_canonical(t.detach().cpu().numpy(), nx, ny, nz, ldx)

    def empty(self, instance):
        import torch
        return torch.zeros(self.layout(instance)[1], dtype=torch.float64, device="cuda")


def gmg_batch_setup(instances, nrhs=1, stream=None) -> GmgBatch:
    return GmgBatch(instances, nrhs, stream)


def gmg_batch_layout(batch, instance):
    return batch.layout(instance)


def gmg_batch_solve(batch, fs, us, rtol=1e-8, maxit=100, stream=None, check=True):
    """fs, us: lists of ninst*nrhs FP64 device tensors (pair i*nrhs + r).
    Returns (iters array, relres array, status)."""
    n = batch.ninst * batch.nrhs
    if len(fs) != n or len(us) != n:
        raise ValueError(f"need {n} right-hand sides and solutions")
    for q in range(n):
        inst = q // batch.nrhs
        elems = batch.layout(inst)[1]
        _field(batch, fs[q], f"f[{q}]", prec=GMG_F64, elems=elems)
        _field(batch, us[q], f"u[{q}]", prec=GMG_F64, elems=elems)
    fp = (C.c_void_p * n)(*[t.data_ptr() for t in fs])
    up = (C.c_void_p * n)(*[t.data_ptr() for t in us])
    it = np.zeros(n, dtype=np.int32)
    rel = np.zeros(n)
    st = _lib.gmg_batch_solve(batch.handle, fp, up, float(rtol), int(maxit),
                              it.ctypes.data_as(C.POINTER(C.c_int)),
                              rel.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream))
    if check and st != GMG_ENOCONV:
        _check(st)
    return it, rel, st


def gmg_setup(**kw) -> GmgContext:
    return GmgContext(**kw)


def gmg_destroy(ctx: GmgContext) -> None:
    ctx.close()


def gmg_field_layout(ctx: GmgContext, level=0):
    return ctx.layout(level)


def _level(ctx, level, lo=0):
    level = int(level)
    if not lo <= level < ctx.nlevels:
        raise ValueError(f"level {level} outside [{lo}, {ctx.nlevels - 1}]")
    return level


def spmv(ctx, level, x, y, stream=None):
    level = _level(ctx, level)
    prec = _fields(ctx, [(x, "x", level), (y, "y", level)])
    _distinct(x, y, "x and y")
    _check(_lib.spmv(ctx.handle, level, prec, _ptr(x), _ptr(y), _stream(stream)))


def line_solve(ctx, level, r, z, stream=None):
    level = _level(ctx, level)
    prec = _fields(ctx, [(r, "r", level), (z, "z", level)])
    _check(_lib.line_solve(ctx.handle, level, prec, _ptr(r), _ptr(z), _stream(stream)))


def line_smooth(ctx, level, f, u, nsweeps=1, rho=None, stream=None):
    level = _level(ctx, level)
    prec = _fields(ctx, [(f, "f", level), (u, "u", level)])
    rho = ctx.rho if rho is None else float(rho)
    _check(_lib.line_smooth(ctx.handle, level, prec, _ptr(f), _ptr(u), int(nsweeps), rho,
                            _stream(stream)))


def gmg_residual(ctx, level, f, u, r, norm=False, stream=None):
    level = _level(ctx, level)
    prec = _fields(ctx, [(f, "f", level), (u, "u", level), (r, "r", level)])
    out = C.c_double()
    _check(_lib.gmg_residual(ctx.handle, level, prec, _ptr(f), _ptr(u), _ptr(r),
                             C.byref(out) if norm else None, _stream(stream)))
    return out.value if norm else None


def gmg_residual_noalloc(ctx, level, f, u, r, norm2=None, stream=None):
    """r = f - A u like gmg_residual, allocating nothing and never
    synchronising: ||r||^2 (FP64) goes to the device tensor `norm2` (float64,
    at least one element) when given, the partial sums to the library's static
    per-GPU scratch.  Calls that overlap on one GPU race."""
    import torch
    level = _level(ctx, level)
    prec = _fields(ctx, [(f, "f", level), (u, "u", level), (r, "r", level)])
    _distinct(r, u, "r and u")
    _distinct(r, f, "r and f")
    out = None
    if norm2 is not None:
        if not isinstance(norm2, torch.Tensor) or norm2.dtype != torch.float64 \
                or not norm2.is_cuda or not norm2.is_contiguous() or norm2.numel() < 1:
            raise ValueError("norm2: expected a contiguous float64 GPU tensor of at least one "
                             "element")
        dev = getattr(ctx, "device", None)
        if dev is not None and norm2.device.index != dev:
            raise ValueError(f"norm2: on cuda:{norm2.device.index}, the context lives on "
                             f"cuda:{dev}")
        out = _ptr(norm2)
    _check(_lib.gmg_residual_noalloc(ctx.handle, level, prec, _ptr(f), _ptr(u), _ptr(r), out,
                                     _stream(stream)))


def gmg_restrict_smooth(ctx, level, rf, fc, uc, rho=None, stream=None):
    level = _level(ctx, level, lo=1)
    prec = _fields(ctx, [(rf, "rf", level - 1), (fc, "fc", level), (uc, "uc", level)])
    rho = ctx.rho if rho is None else float(rho)
    _check(_lib.gmg_restrict_smooth(ctx.handle, level, prec, _ptr(rf), _ptr(fc),
                                    _ptr(uc), rho, _stream(stream)))


def gmg_prolongate(ctx, level, uc, uf, stream=None):
    level = _level(ctx, level, lo=1)
    prec = _fields(ctx, [(uc, "uc", level), (uf, "uf", level - 1)])
    _check(_lib.gmg_prolongate(ctx.handle, level, prec, _ptr(uc), _ptr(uf),
                               _stream(stream)))


def gmg_vcycle(ctx, f, u, stream=None):
    _fields(ctx, [(f, "f", 0), (u, "u", 0)], prec=ctx.prec_precond)
    _check(_lib.gmg_vcycle(ctx.handle, _ptr(f), _ptr(u), _stream(stream)))


def gmg_solve(ctx, f, u, rtol=1e-8, maxit=100, stream=None, check=True):
    """Returns (iters, relres, history, status)."""
    _fields(ctx, [(f, "f", 0), (u, "u", 0)], prec=GMG_F64)
    it, rel = C.c_int(), C.c_double()
    hist = np.zeros(maxit + 1)
    st = _lib.gmg_solve(ctx.handle, _ptr(f), _ptr(u), float(rtol), int(maxit), C.byref(it),
                        C.byref(rel), hist.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream))
    if check and st != GMG_ENOCONV:
        _check(st)
    return it.value, rel.value, hist[: it.value + 1].copy(), st


def pcg_solve(ctx, f, u, rtol=1e-8, maxit=1000, precond=0, stream=None, check=True):
    """Returns (iters, true relres, recursive history, status)."""
    _fields(ctx, [(f, "f", 0), (u, "u", 0)], prec=GMG_F64)
    it, rel = C.c_int(), C.c_double()
    hist = np.zeros(maxit + 1)
    st = _lib.pcg_solve(ctx.handle, _ptr(f), _ptr(u), float(rtol), int(maxit), int(precond),
                        C.byref(it), C.byref(rel), hist.ctypes.data_as(C.POINTER(C.c_double)),
                        _stream(stream))
    if check and st != GMG_ENOCONV:
        _check(st)
    return it.value, rel.value, hist[: it.value + 1].copy(), st


def gmg_timing_enable(ctx, enable=True):
    _check(_lib.gmg_timing_enable(ctx.handle, 1 if enable else 0))


def gmg_timing_filter(ctx, kernels=None):
    """Time only the given kernel kinds (names or ids); None times every kind."""
    mask = 0xFFFFFFFF
    if kernels is not None:
        mask = 0
        for k in kernels:
            mask |= 1 << (KERNELS.index(k) if isinstance(k, str) else int(k))
    _check(_lib.gmg_timing_filter(ctx.handle, C.c_uint32(mask)))


def gmg_timing_read(ctx, kernel, level=-1, prec=GMG_F64):
    """(launch count, total ms) of one kernel kind since timing was enabled."""
    if isinstance(kernel, str):
        kernel = KERNELS.index(kernel)
    n, ms = C.c_int64(), C.c_double()
    _check(_lib.gmg_timing_read(ctx.handle, int(kernel), int(level), int(prec), C.byref(n),
                                C.byref(ms)))
    return n.value, ms.value


def gmg_timing_table(ctx):
    """{(kernel, level, prec): (count, ms)} for every kernel that ran."""
    out = {}
    for kid, name in enumerate(KERNELS):
        for lvl in range(ctx.nlevels):
            for prec in (GMG_F64, GMG_F32):
                n, ms = gmg_timing_read(ctx, kid, lvl, prec)
                if n:
                    out[(name, lvl, "f64" if prec == GMG_F64 else "f32")] = (n, ms)
    return out


def gmg_last_error() -> str:
    return _lib.gmg_last_error().decode()


# ---------------------------------------------------------------------------
# Launch shapes (per kernel kind, level and precision) and the autotuner
# ---------------------------------------------------------------------------
# kernel kinds whose launch shape the solvers use
TUNED_KERNELS = ("spmv", "residual", "line_solve", "smooth", "prolongate", "cg_spmv",
                 "cg_tridiag", "correct", "fcg", "residual_restrict", "prolong_smooth")
LAUNCH_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "launch_shapes.json")


def _kid(kernel):
    return KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)


def gmg_set_launch(ctx, kernel, level, prec, rows, group):
    _check(_lib.gmg_set_launch(ctx.handle, _kid(kernel), int(level), int(prec), int(rows),
                               int(group)))


def gmg_get_launch(ctx, kernel, level, prec):
    rows, group = C.c_int(), C.c_int()
    _check(_lib.gmg_get_launch(ctx.handle, _kid(kernel), int(level), int(prec), C.byref(rows),
                               C.byref(group)))
    return rows.value, group.value


def gmg_set_graphs(ctx, enable=True):
    """Iterations of the solvers as hipGraph replays (True, the default) or
    as direct launches (False); results are identical."""
    _check(_lib.gmg_set_graphs(ctx.handle, 1 if enable else 0))


def gmg_solver_polls(ctx):
    """Host waits for device scalars in the context's last solve."""
    return _check(_lib.gmg_solver_polls(ctx.handle))


def gmg_autotune(ctx, reps=3, stream=None):
    """Time every candidate launch shape of every kernel the solvers use and keep
    the fastest (overwrites the context's work buffers; synchronises)."""
    _check(_lib.gmg_autotune(ctx.handle, int(reps), _stream(stream)))


def launch_table(ctx):
    """{"kernel/level/prec": [rows, group]} for every tuned kernel kind."""
    out = {}
    for k in TUNED_KERNELS:
        for lvl in range(ctx.nlevels):
            for prec in (GMG_F64, GMG_F32):
                out[f"{k}/{lvl}/{prec}"] = list(gmg_get_launch(ctx, k, lvl, prec))
    return out


def apply_launch_table(ctx, table):
    for key, (rows, group) in table.items():
        k, lvl, prec = key.split("/")
        if int(lvl) < ctx.nlevels:
            gmg_set_launch(ctx, k, int(lvl), int(prec), rows, group)


def launch_key(ctx):
    """Key of a context's tuned shapes: device, grid, levels and preconditioner
    precision."""
    import torch
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", dev.name).split(":")[0]
    return f"{arch}|{ctx.nx}x{ctx.ny}x{ctx.nz}|L{ctx.nlevels}|p{ctx.prec_precond}"


def tuned(ctx, reps=3, path=LAUNCH_TABLE, stream=None):
    """Apply the stored launch shapes for this context's key, or run the
    autotuner and return the new table.  Returns (table, from_store)."""
    import json
    key = launch_key(ctx)
    store = {}
    if path and os.path.exists(path):
        with open(path) as fh:
            store = json.load(fh)
    if key in store:
        apply_launch_table(ctx, store[key])
        return store[key], True
    gmg_autotune(ctx, reps, stream)
    return launch_table(ctx), False


# ---------------------------------------------------------------------------
# Layout conversion and host-memory solves
# ---------------------------------------------------------------------------
def gmg_copy_probe(src, dst, stream=None):
    """Plain streaming copy of a device tensor into another of the same size
    (the bandwidth ceiling the kernels are judged against)."""
    import torch
    for t, name in ((src, "src"), (dst, "dst")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous GPU tensor")
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("src and dst must have the same size in bytes")
    if src.numel() == 0:
        return  # (empty tensors carry no device pointer)
    _check(_lib.gmg_copy_probe(src.data_ptr(), dst.data_ptr(),
                               src.numel() * src.element_size(), _stream(stream)))


def _canonical_elems(ctx, level):
    nx, ny, nz = ctx.shape(level)
    return nx * ny * nz


def gmg_transpose_in(ctx, level, src_z, dst_x, stream=None):
    """Device z-contiguous (j*nx+i)*nz+k -> x-contiguous field (same dtype)."""
    level = _level(ctx, level)
    prec = _field(ctx, src_z, "src_z", level, elems=_canonical_elems(ctx, level))
    _field(ctx, dst_x, "dst_x", level, prec)
    _distinct(src_z, dst_x, "src_z and dst_x")
    _check(_lib.gmg_transpose_in(ctx.handle, level, prec, src_z.data_ptr(),
                                 dst_x.data_ptr(), _stream(stream)))


def gmg_transpose_out(ctx, level, src_x, dst_z, stream=None):
    """Device x-contiguous field -> z-contiguous (j*nx+i)*nz+k (same dtype)."""
    level = _level(ctx, level)
    prec = _field(ctx, src_x, "src_x", level)
    _field(ctx, dst_z, "dst_z", level, prec, elems=_canonical_elems(ctx, level))
    _distinct(src_x, dst_z, "src_x and dst_z")
    _check(_lib.gmg_transpose_out(ctx.handle, level, prec, src_x.data_ptr(),
                                  dst_z.data_ptr(), _stream(stream)))


HOST_METHODS = {"mg": 0, "pcg": 1, "fcg": 2}


def gmg_solve_host(ctx, f, u, method="mg", rtol=1e-8, maxit=100, stream=None, check=True):
    """Solve from host arrays in canonical z-contiguous order (FP64, C order);
    u is the initial guess and is overwritten with the solution.  Returns
    (iters, relres, timings_ms dict, status)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.flags.c_contiguous):
        raise ValueError("u must be a C-contiguous float64 numpy array (it is overwritten)")
    n = ctx.nx * ctx.ny * ctx.nz
    if f.size != n or u.size != n:
        raise ValueError(f"f and u need {n} values")
    it, rel = C.c_int(), C.c_double()
    tm = (C.c_double * 5)()
    m = HOST_METHODS[method] if isinstance(method, str) else int(method)
    st = _lib.gmg_solve_host(ctx.handle, m, f.ctypes.data_as(C.c_void_p),
                             u.ctypes.data_as(C.c_void_p), float(rtol), int(maxit), C.byref(it),
                             C.byref(rel), tm, _stream(stream))
    if check and st != GMG_ENOCONV:
        _check(st)
    names = ("copy_in", "layout_in", "solve", "layout_out", "copy_out")
    return it.value, rel.value, dict(zip(names, list(tm))), st
