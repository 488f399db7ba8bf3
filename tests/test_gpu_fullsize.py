"""Full-size parity: the 1024 x 1024 x 128 grid of one GPU's share (K_T ~
U[0.5,2], K_v = 1e4, 6 levels), in the same launch configuration the benchmark
times.  The oracle cannot assemble this operator in a test, so it checks the
GPU outputs at sampled columns (all layers) with its row-wise forms, and the
solver result through the FP64 residual norm over all rows."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import device_index, max_rel, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NCOLS = 512


@pytest.fixture(scope="module")
def share():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1402_3545_amd as G
    w = W.SHARE
    ctx, orc, kh = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                           kh_model=w.kh_model, matfree=True)
    G.tuned(ctx)      # the benchmark's stored launch shapes
    rng = np.random.default_rng(1234)
    cols = np.unique(np.concatenate([
        rng.integers(0, w.nx * w.ny, NCOLS),
        [0, w.nx - 1, w.nx * (w.ny - 1), w.nx * w.ny - 1]]))      # wrap-around corners
    return w, ctx, orc, cols


def _gather(ctx, t, rows, level=0):
    idx = device_index(ctx, rows, level)
    # host-side bounds check before the device gather
    assert idx.size and idx.min() >= 0 and idx.max() < t.numel(), (idx.min(), idx.max(), t.numel())
    return t.index_select(0, torch.from_numpy(idx).cuda()).double().cpu().numpy()


def test_fullsize_kernels_at_sampled_columns(share):
    import paper_1402_3545_amd as G
    w, ctx, orc, cols = share
    n = w.unknowns
    x = W.uniform_pm1(77, 1, n)
    f = w.rhs()
    rows = orc.column_rows(cols)
    xd, fd, yd = ctx.to_device(x), ctx.to_device(f), ctx.empty()
    # SpMV
    G.spmv(ctx, 0, xd, yd)
    ref = orc.apply_rows(rows, x)
    scale = np.abs(ref).max()
    assert max_rel(_gather(ctx, yd, rows), ref, scale) < 1e-12
    # residual
    G.gmg_residual(ctx, 0, fd, xd, yd)
    rref = f[rows] - ref
    assert max_rel(_gather(ctx, yd, rows), rref, np.abs(rref).max()) < 1e-12
    # line solve
    G.line_solve(ctx, 0, fd, yd)
    zref = orc.line_solve_columns(cols, f)[rows]
    assert max_rel(_gather(ctx, yd, rows), zref, np.abs(zref).max()) < 1e-12
    # smooth: u + rho M^-1 (f - A u) on the sampled columns
    ud = xd.clone()
    G.line_smooth(ctx, 0, fd, ud)
    r_full = np.zeros(n)
    r_full[rows] = f[rows] - ref
    sref = x[rows] + ctx.rho * orc.line_solve_columns(cols, r_full)[rows]
    assert max_rel(_gather(ctx, ud, rows), sref, np.abs(sref).max()) < 1e-12


def test_fullsize_transfers_at_sampled_columns(share):
    import paper_1402_3545_amd as G
    w, ctx, orc, cols = share
    n = w.unknowns
    rf = W.uniform_pm1(78, 1, n)
    nc = orc.size(1)
    rfd = ctx.to_device(rf)
    fcd, ucd = ctx.empty(1), ctx.empty(1)
    G.gmg_restrict_smooth(ctx, 1, rfd, fcd, ucd)
    fc_ref = orc.restrict(rf, 0)
    ncx = w.nx // 2
    ccols = np.unique((cols // w.nx // 2) * ncx + (cols % w.nx) // 2)   # parents (I, J)
    assert ccols.max() < ncx * (w.ny // 2)
    crow = orc.column_rows(ccols)
    assert max_rel(_gather(ctx, fcd, crow, 1), fc_ref[crow], np.abs(fc_ref).max()) < 1e-12
    uc_ref = ctx.rho * orc.line_solve_columns(ccols, fc_ref, depth=1)[crow]
    assert max_rel(_gather(ctx, ucd, crow, 1), uc_ref, np.abs(uc_ref).max()) < 1e-12
    uc = W.uniform_pm1(79, 1, nc)
    ufd = ctx.to_device(rf)
    G.gmg_prolongate(ctx, 1, ctx.to_device(uc, 1), ufd)
    pref = orc.prolongate_add(uc, rf, 1)
    rows = orc.column_rows(cols)
    assert max_rel(_gather(ctx, ufd, rows), pref[rows], np.abs(pref).max()) < 1e-12


def test_fullsize_mg_solve_true_residual(share):
    import paper_1402_3545_amd as G
    w, ctx, orc, _ = share
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=w.rtol, maxit=60)
    assert st == 0 and 5 < it < 40
    assert (np.diff(hist) < 0).all()
    u = ctx.from_device(ud)
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < w.rtol
    assert true_rel == pytest.approx(rel, rel=1e-6)


def test_fullsize_pcg_true_residual(share):
    """The fused line-PCG of the benchmark (its stored launch shapes) on the
    full share: FP64 true residual over all rows below the tolerance."""
    import paper_1402_3545_amd as G
    w, ctx, orc, _ = share
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=w.rtol, maxit=2000)
    assert st == 0 and 20 < it < 400
    true_rel = orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1.01 * w.rtol
    assert true_rel == pytest.approx(rel, rel=1e-6)


@pytest.mark.parametrize("method", ["refinement", "fcg_vcycle", "fcg_line"])
def test_fullsize_mixed_precision_true_residual(share, method):
    """The FP32-preconditioned solvers of the benchmark on the full share, in
    its stored launch shapes: FP64 true residual over all rows."""
    import paper_1402_3545_amd as G
    w, ctx, orc, _ = share
    ctx32 = G.GmgContext(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=1.0, zfaces=w.zfaces(),
                         kh=W.kh_uniform(w.seed, w.nx, w.ny), prec_precond=G.GMG_F32)
    G.tuned(ctx32)
    f = w.rhs()
    fd, ud = ctx32.to_device(f), ctx32.empty()
    if method == "refinement":
        it, rel, _, st = G.gmg_solve(ctx32, fd, ud, rtol=w.rtol, maxit=60)
    else:
        it, rel, _, st = G.pcg_solve(ctx32, fd, ud, rtol=w.rtol, maxit=2000,
                                     precond=1 if method == "fcg_vcycle" else 2)
    assert st == 0
    true_rel = orc.residual_norm2_rows(f, ctx32.from_device(ud)) ** 0.5 / np.linalg.norm(f)
    assert true_rel < w.rtol
    assert true_rel == pytest.approx(rel, rel=1e-5)
    ctx32.close()
