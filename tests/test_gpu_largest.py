"""Full-size parity on the largest single-GPU grid: 2048 x 2048 x 128 =
536,870,912 unknowns, K_T = exp(0.5 N(0,1)) per column, K_v = 1e5, 7 levels,
tolerance 1e-8.  Both the FP64 multigrid solve and the mixed-precision one
(FP32 V-cycles inside FP64 iterative refinement) run on the device; the oracle
(matrix-free row-wise form, no CSR) computes the FP64 true residual of each
solution over every row, and the kernels' outputs at sampled columns."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import device_index, max_rel, problem

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")

NCOLS = 256


@pytest.fixture(scope="module")
def largest():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1402_3545_amd as G
    w = W.LARGEST
    ctx, orc, kh = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                           kh_model=w.kh_model, matfree=True)
    ctx32 = G.GmgContext(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=1.0, zfaces=w.zfaces(),
                         kh=kh, prec_precond=G.GMG_F32)
    for c in (ctx, ctx32):
        G.tuned(c)    # the benchmark's stored launch shapes
    f = w.rhs()
    fd = ctx.to_device(f)
    yield w, ctx, ctx32, orc, f, fd
    del fd
    ctx32.close()
    ctx.close()
    torch.cuda.empty_cache()


def _gather(ctx, t, rows, level=0):
    idx = device_index(ctx, rows, level)
    assert idx.size and idx.min() >= 0 and idx.max() < t.numel(), (idx.min(), idx.max(), t.numel())
    return t.index_select(0, torch.from_numpy(idx).cuda()).double().cpu().numpy()


def test_largest_kernels_at_sampled_columns(largest):
    import paper_1402_3545_amd as G
    w, ctx, _, orc, f, fd = largest
    rng = np.random.default_rng(4321)
    cols = np.unique(np.concatenate([rng.integers(0, w.nx * w.ny, NCOLS),
                                     [0, w.nx - 1, w.nx * (w.ny - 1), w.nx * w.ny - 1]]))
    rows = orc.column_rows(cols)
    yd = ctx.empty()
    G.spmv(ctx, 0, fd, yd)
    ref = orc.apply_rows(rows, f)
    assert max_rel(_gather(ctx, yd, rows), ref, np.abs(ref).max()) < 1e-12
    G.line_solve(ctx, 0, fd, yd)
    zref = orc.line_solve_columns(cols, f)[rows]
    assert max_rel(_gather(ctx, yd, rows), zref, np.abs(zref).max()) < 1e-12
    del yd


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_largest_mg_solve_true_residual(largest, prec):
    import paper_1402_3545_amd as G
    w, ctx, ctx32, orc, f, fd = largest
    c = ctx if prec == "f64" else ctx32
    ud = ctx.empty()
    it, rel, hist, st = G.gmg_solve(c, fd, ud, rtol=w.rtol, maxit=80)
    assert st == 0, G.gmg_last_error()
    assert 5 < it < 60
    assert (np.diff(hist[:it + 1]) < 0).all()
    u = ctx.from_device(ud)
    del ud
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < w.rtol
    assert true_rel == pytest.approx(rel, rel=1e-6)
