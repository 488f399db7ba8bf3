"""Parity of every HIP kernel with the CPU oracle, element by element.

FP64 bar: 1e-12 relative.  For the stencil kernels the error of a row is
measured against |A||x| (+|f|), the size of the terms that are summed, so that
cancellation cannot fake a failure; for the line kernels against max|z|
(the column systems have Skeel condition numbers of a few tens, so two stable
eliminations agree to ~1e-15).

FP32 bars: inputs are rounded to FP32 before both sides see them; the
oracle computes in FP64.  Stencils: coefficients rounded to FP32 (relative
6e-8) and a 7-term sum give 2e-6, scaled as above.  Line kernels: the error of
an FP32 elimination grows with the column height (a textbook FP32 Thomas sweep
on the FP32-rounded columns of these operators is off by 2.3e-5 of max|z| at
n_z = 128 and 4e-6 at n_z = 64), so the bar is 4e-7 n_z (about seven FP32
unit roundoffs per layer), at least 2e-6.
"""

import ctypes as C

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import abs_matvec, f32_line_bar, max_rel, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [
    (4, 4, 8),        # tiny
    (40, 6, 37),      # ragged width (padding), odd nz, partial tiles
    (64, 64, 64),     # the small workload's grid: many tiles
    (96, 32, 2),      # minimum nz
    (34, 10, 128),    # maximum nz, ragged
    (16, 18, 127),    # odd maximum
    (192, 6, 37),     # three full 64-column tiles (east/west by lane shifts, periodic halo)
    (200, 5, 64),     # three full tiles and a ragged one
]
F64 = 1e-12
F32_STENCIL = 2e-6


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _dtype(prec):
    return torch.float64 if prec == 0 else torch.float32


def _inputs(n, seed, prec):
    x = W.uniform_pm1(seed, 1, n)
    f = W.uniform_pm1(seed, 2, n)
    if prec == 1:
        x = x.astype(np.float32).astype(np.float64)
        f = f.astype(np.float32).astype(np.float64)
    return x, f


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_spmv(shape, prec):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz)
    x, _ = _inputs(nx * ny * nz, 11, prec)
    xd = ctx.to_device(x, dtype=_dtype(prec))
    yd = ctx.empty(dtype=_dtype(prec))
    G.spmv(ctx, 0, xd, yd)
    torch.cuda.synchronize()
    got = ctx.from_device(yd)
    ref = orc.spmv(x)
    bar = F64 if prec == 0 else F32_STENCIL
    assert max_rel(got, ref, abs_matvec(orc, x)) < bar


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_residual_and_norm(shape, prec):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, seed=5)
    u, f = _inputs(nx * ny * nz, 12, prec)
    ud, fd = ctx.to_device(u, dtype=_dtype(prec)), ctx.to_device(f, dtype=_dtype(prec))
    rd = ctx.empty(dtype=_dtype(prec))
    nrm2 = G.gmg_residual(ctx, 0, fd, ud, rd, norm=True)
    got = ctx.from_device(rd)
    ref = orc.residual(f, u)
    bar = F64 if prec == 0 else F32_STENCIL
    assert max_rel(got, ref, abs_matvec(orc, u) + np.abs(f)) < bar
    # the norm is accumulated in FP64 from the kernel's own r values
    assert nrm2 == pytest.approx(float(got @ got), rel=1e-12 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_line_solve(shape, prec):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, kv=1e4, seed=6)
    r, _ = _inputs(nx * ny * nz, 13, prec)
    rd = ctx.to_device(r, dtype=_dtype(prec))
    zd = ctx.empty(dtype=_dtype(prec))
    G.line_solve(ctx, 0, rd, zd)
    got = ctx.from_device(zd)
    ref = orc.line_solve(r)
    bar = F64 if prec == 0 else f32_line_bar(nz)
    assert max_rel(got, ref, np.abs(ref).max()) < bar
    # in place (r and z the same buffer) gives the same result
    G.line_solve(ctx, 0, rd, rd)
    assert np.array_equal(ctx.from_device(rd), got)


@pytest.mark.parametrize("nsweeps", [1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_line_smooth(shape, prec, nsweeps):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, seed=7)
    u, f = _inputs(nx * ny * nz, 14, prec)
    ud, fd = ctx.to_device(u, dtype=_dtype(prec)), ctx.to_device(f, dtype=_dtype(prec))
    G.line_smooth(ctx, 0, fd, ud, nsweeps=nsweeps)
    got = ctx.from_device(ud)
    ref = u.copy()
    for _ in range(nsweeps):
        ref = orc.smooth(f, ref)
    bar = F64 if prec == 0 else f32_line_bar(nz)
    assert max_rel(got, ref, np.abs(ref).max()) < bar * nsweeps


MULTI = [((8, 8, 4), 2), ((64, 64, 64), 4), ((40, 24, 37), 3), ((32, 96, 128), 2)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,L", MULTI)
def test_restrict_smooth(shape, L, prec):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, nlevels=L, seed=8)
    for lvl in range(1, L):
        rf, _ = _inputs(orc.size(lvl - 1), 15 + lvl, prec)
        rfd = ctx.to_device(rf, lvl - 1, dtype=_dtype(prec))
        fcd, ucd = ctx.empty(lvl, dtype=_dtype(prec)), ctx.empty(lvl, dtype=_dtype(prec))
        G.gmg_restrict_smooth(ctx, lvl, rfd, fcd, ucd)
        fc_ref, uc_ref = orc.restrict_smooth(rf, lvl)
        bar = F64 if prec == 0 else f32_line_bar(nz)
        assert max_rel(ctx.from_device(fcd, lvl), fc_ref, np.abs(fc_ref).max()) < bar
        assert max_rel(ctx.from_device(ucd, lvl), uc_ref, np.abs(uc_ref).max()) < bar


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,L", MULTI)
def test_prolongate(shape, L, prec):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, nlevels=L, seed=9)
    for lvl in range(1, L):
        uc, _ = _inputs(orc.size(lvl), 20 + lvl, prec)
        uf, _ = _inputs(orc.size(lvl - 1), 30 + lvl, prec)
        ucd = ctx.to_device(uc, lvl, dtype=_dtype(prec))
        ufd = ctx.to_device(uf, lvl - 1, dtype=_dtype(prec))
        G.gmg_prolongate(ctx, lvl, ucd, ufd)
        ref = orc.prolongate_add(uc, uf, lvl)
        bar = F64 if prec == 0 else F32_STENCIL
        assert max_rel(ctx.from_device(ufd, lvl - 1), ref, np.abs(ref).max()) < bar


def test_kernels_are_deterministic():
    import paper_1402_3545_amd as G
    ctx, orc, _ = problem(64, 64, 64, nlevels=4)
    u, f = _inputs(64 ** 3, 40, 0)
    ud, fd = ctx.to_device(u), ctx.to_device(f)
    rd = ctx.empty()
    n1 = G.gmg_residual(ctx, 0, fd, ud, rd, norm=True)
    n2 = G.gmg_residual(ctx, 0, fd, ud, rd, norm=True)
    assert n1 == n2
    a, b = ud.clone(), ud.clone()
    G.gmg_vcycle(ctx, fd, a)
    G.gmg_vcycle(ctx, fd, b)
    assert torch.equal(a, b)


def test_invalid_arguments_raise():
    import paper_1402_3545_amd as G
    ctx, _, _ = problem(8, 8, 4, nlevels=2)
    x = ctx.empty()
    y = ctx.empty()
    # the binding rejects them before the call ...
    with pytest.raises(ValueError):
        G.spmv(ctx, 2, x, y)                      # no such level
    with pytest.raises(ValueError):
        G.spmv(ctx, 0, x, x)                      # aliasing
    with pytest.raises(ValueError):
        G.gmg_restrict_smooth(ctx, 0, x, x, x)    # level 0 is not coarse
    with pytest.raises(ValueError):
        G.gmg_solve(ctx, x.float(), y)            # FP32 field in an FP64 solve
    with pytest.raises(G.GmgError):
        G.gmg_solve(ctx, x, x)                    # f and u overlap
    # ... and the C ABI itself validates what it can see
    px, py, h = C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), ctx.handle
    assert G._lib.spmv(h, 2, G.GMG_F64, px, py, None) == G.GMG_EINVAL
    assert G._lib.spmv(h, 0, G.GMG_F64, px, px, None) == G.GMG_EINVAL
    assert G._lib.gmg_restrict_smooth(h, 0, G.GMG_F64, px, px, px, 0.5, None) == G.GMG_EINVAL


def _pcr_everywhere(G, ctx):
    for lvl in range(ctx.nlevels):
        for prec in (G.GMG_F64, G.GMG_F32):
            G.gmg_set_launch(ctx, "line_solve", lvl, prec, 1, 0)
            G.gmg_set_launch(ctx, "smooth", lvl, prec, 1, 0)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_line_kernels_by_cyclic_reduction(shape, prec):
    """One wavefront per column, parallel cyclic reduction (the coarse-level
    launch shape): same bars against the oracle as the twisted elimination."""
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, kv=1e4, seed=6)
    _pcr_everywhere(G, ctx)
    r, f = _inputs(nx * ny * nz, 13, prec)
    rd = ctx.to_device(r, dtype=_dtype(prec))
    zd = ctx.empty(dtype=_dtype(prec))
    G.line_solve(ctx, 0, rd, zd)
    ref = orc.line_solve(r)
    bar = F64 if prec == 0 else f32_line_bar(nz)
    assert max_rel(ctx.from_device(zd), ref, np.abs(ref).max()) < bar
    ud, fd = ctx.to_device(r, dtype=_dtype(prec)), ctx.to_device(f, dtype=_dtype(prec))
    G.line_smooth(ctx, 0, fd, ud, nsweeps=2)
    sref = orc.smooth(f, orc.smooth(f, r))
    assert max_rel(ctx.from_device(ud), sref, np.abs(sref).max()) < 2 * bar


@pytest.mark.parametrize("bc_h", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", SHAPES + [(2, 2, 8), (3, 3, 5), (65, 9, 3)])
def test_line_smooth_with_staged_neighbours(shape, prec, bc_h):
    """The smoother with its horizontal neighbours staged in LDS by the
    workgroup (launch shape rows = 2): same bars as the per-lane loads, also
    on grids narrower than a tile, with walls, and (2 x 2 grids) on a coarse
    level of a single column."""
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    one_col = (nx, ny) == (2, 2)
    L = 2 if one_col else 1
    lvl = L - 1
    ctx, orc, _ = problem(nx, ny, nz, nlevels=L, seed=7, bc_h=bc_h)
    for p in (G.GMG_F64, G.GMG_F32):
        G.gmg_set_launch(ctx, "smooth", lvl, p, 2, 0)
    n = (nx >> lvl) * (ny >> lvl) * nz
    u, f = _inputs(n, 14, prec)
    ud = ctx.to_device(u, lvl, dtype=_dtype(prec))
    fd = ctx.to_device(f, lvl, dtype=_dtype(prec))
    G.line_smooth(ctx, lvl, fd, ud, nsweeps=2)
    ref = orc.smooth(f, orc.smooth(f, u, depth=lvl), depth=lvl)
    bar = F64 if prec == 0 else f32_line_bar(nz)
    assert max_rel(ctx.from_device(ud, lvl), ref, np.abs(ref).max()) < 2 * bar
