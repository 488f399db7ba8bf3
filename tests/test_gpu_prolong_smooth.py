"""The V-cycle's prolongation folded into the staged post-smoother.

The folded kernel adds the same 9/3/3/1 correction, with the same arithmetic,
to every value the smoother stages, instead of storing u + P u_c first; the
V-cycle must therefore give the same result as with the two kernels, and
match the oracle's V-cycle like every other launch shape."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import problem, max_rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _fold(G, ctx, on, group=0):
    """on: False (two kernels), True or 2 (folded, one wavefront per column),
    3 (folded, two wavefronts per column where the level fits)."""
    rows = 4 if not on else (3 if on == 3 else 2)
    for lvl in range(ctx.nlevels):
        for prec in (G.GMG_F64, G.GMG_F32):
            G.gmg_set_launch(ctx, "prolong_smooth", lvl, prec, rows, group if on else 0)


# grids: full 32-column tiles, ragged tiles and odd n_z, n_x below one tile,
# a coarsest level of one column, and the 128-layer columns of the benchmark
GRIDS = [((64, 64, 64), 3), ((96, 40, 37), 3), ((136, 12, 20), 3), ((8, 8, 9), 3),
         ((2, 2, 9), 2), ((32, 64, 128), 4), ((256, 12, 128), 3), ((128, 64, 32), 2)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("bc_h", [0, 1])
@pytest.mark.parametrize("grid", GRIDS)
def test_vcycle_folded_equals_separate_and_oracle(grid, bc_h, prec):
    import paper_1402_3545_amd as G
    (nx, ny, nz), L = grid
    ctx, orc, _ = problem(nx, ny, nz, nlevels=L, seed=61, bc_h=bc_h, prec_precond=prec)
    n = nx * ny * nz
    f, u = W.uniform_pm1(61, 1, n), W.uniform_pm1(61, 2, n)
    dt = torch.float64 if prec == 0 else torch.float32
    if prec == 1:
        f = f.astype(np.float32).astype(np.float64)
        u = u.astype(np.float32).astype(np.float64)
    fd = ctx.to_device(f, dtype=dt)
    outs = []
    for on, group in ((False, 0), (True, 0), (True, 2), (3, 0), (3, 4)):
        _fold(G, ctx, on, group)
        ud = ctx.to_device(u, dtype=dt)
        G.gmg_vcycle(ctx, fd, ud)
        outs.append(ctx.from_device(ud))
    ref = orc.vcycle(f, u)
    scale = np.abs(ref).max()
    # the same arithmetic (the correction's multiply-adds are spelled out in
    # one helper both kernels call): bitwise equal, in any tile order
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert max_rel(outs[1], ref, scale) < (1e-11 if prec == 0 else 1e-4)


@pytest.mark.parametrize("bc_h", [0, 1])
def test_mg_solve_with_folded_prolongation_matches_oracle(bc_h):
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, bc_h=bc_h)
    f = w.rhs()
    fd = ctx.to_device(f)
    res = []
    for on in (False, True):
        _fold(G, ctx, on)
        ud = ctx.empty()
        it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-10, maxit=60)
        assert st == 0
        res.append((it, hist, ctx.from_device(ud)))
    (it0, h0, u0), (it1, h1, u1) = res
    u_ref, it_ref, hist_ref, st_ref = orc.mg_solve(f, rtol=1e-10, maxit=60)
    assert st_ref == 0 and it1 == it0 == it_ref
    # atol: the last cycles' relative residuals sit near the rounding floor
    np.testing.assert_allclose(h1, hist_ref, rtol=1e-9, atol=1e-14)
    assert max_rel(u1, u_ref, np.abs(u_ref).max()) < 1e-9
    true_rel = orc.residual_norm2_rows(f, u1) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-10


def test_folded_prolongation_in_mixed_and_flexible_solves():
    """FP32 V-cycles with the folded prolongation inside FP64 refinement and
    flexible CG reach the FP64 tolerance with the same cycle counts."""
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=1)
    f = w.rhs()
    fd = ctx.to_device(f)
    counts = []
    for on in (False, True):
        _fold(G, ctx, on)
        ud = ctx.empty()
        it, rel, _, st = G.gmg_solve(ctx, fd, ud, rtol=1e-10, maxit=60)
        assert st == 0
        assert orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f) < 1e-10
        ud.zero_()
        itf, relf, _, stf = G.pcg_solve(ctx, fd, ud, rtol=1e-10, maxit=60, precond=1)
        assert stf == 0
        assert orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f) < 1e-10
        counts.append((it, itf))
    assert counts[0] == counts[1]


def test_folded_prolongation_launch_validation():
    import paper_1402_3545_amd as G
    ctx, _, _ = problem(16, 16, 8, nlevels=2)
    assert G.gmg_get_launch(ctx, "prolong_smooth", 0, G.GMG_F64) == (4, 0)  # off by default
    G.gmg_set_launch(ctx, "prolong_smooth", 0, G.GMG_F64, 2, 4)
    assert G.gmg_get_launch(ctx, "prolong_smooth", 0, G.GMG_F64) == (2, 4)
    for rows in (1, 8, 16, 0):
        with pytest.raises(G.GmgError):
            G.gmg_set_launch(ctx, "prolong_smooth", 0, G.GMG_F64, rows, 0)
