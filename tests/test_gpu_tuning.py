"""Launch shapes and the autotuner: every shape computes the same values.

The stencil and line kernels compute each output element with the same
arithmetic whatever the workgroup shape and tile order, so their outputs must
be bitwise identical across shapes; only FP64 reductions (norms, dot products)
may differ, in their summation order.  After autotuning, the solvers still
match the oracle."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(4, 0), (8, 0), (16, 0), (4, 1), (8, 2), (16, 4), (4, 8)]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _set_all(G, ctx, rows, group):
    for k in G.TUNED_KERNELS:
        if k == "prolong_smooth":  # a V-cycle choice (rows 4 or 2), not a tiling
            continue
        for lvl in range(ctx.nlevels):
            for prec in (G.GMG_F64, G.GMG_F32):
                G.gmg_set_launch(ctx, k, lvl, prec, rows, group)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("grid", [(96, 40, 37, 3), (256, 24, 64, 2)])
def test_kernels_bitwise_identical_across_shapes(grid, prec):
    import paper_1402_3545_amd as G
    nx, ny, nz, L = grid
    ctx, _, _ = problem(nx, ny, nz, nlevels=L, seed=21)
    dt = torch.float64 if prec == 0 else torch.float32
    n = nx * ny * nz
    x = ctx.to_device(W.uniform_pm1(31, 1, n), dtype=dt)
    f = ctx.to_device(W.uniform_pm1(31, 2, n), dtype=dt)
    ref = None
    for rows, group in SHAPES:
        _set_all(G, ctx, rows, group)
        y, r, u = ctx.empty(dtype=dt), ctx.empty(dtype=dt), x.clone()
        G.spmv(ctx, 0, x, y)
        nrm = G.gmg_residual(ctx, 0, f, x, r, norm=True)
        G.line_smooth(ctx, 0, f, u, nsweeps=2)
        uc = ctx.to_device(W.uniform_pm1(32, 1, (nx // 2) * (ny // 2) * nz), 1, dtype=dt)
        uf = x.clone()
        G.gmg_prolongate(ctx, 1, uc, uf)
        out = [t.cpu() for t in (y, r, u, uf)]
        if ref is None:
            ref, ref_nrm = out, nrm
            continue
        for a, b in zip(out, ref):
            assert torch.equal(a, b), (rows, group)
        assert nrm == pytest.approx(ref_nrm, rel=1e-13 if prec == 0 else 1e-12)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("grid", [(40, 6, 37), (64, 64, 64), (34, 10, 128), (2, 2, 9),
                                  (128, 6, 128), (192, 2, 32), (64, 4, 64)])
def test_staged_smoother_bitwise_equal_to_per_lane_loads(grid, prec):
    """Staging the neighbours in LDS (rows = 2), also with the two halves of a
    column in two wavefronts (rows = 3: nx a multiple of 64, ny even, 32, 64 or
    128 layers; elsewhere it runs as rows = 2), changes where the values come
    from, not the arithmetic: the smoother's output is bitwise identical."""
    import paper_1402_3545_amd as G
    nx, ny, nz = grid
    dt = torch.float64 if prec == 0 else torch.float32
    outs = []
    for rows in (4, 2, 3):
        ctx, _, _ = problem(nx, ny, nz, seed=22)
        G.gmg_set_launch(ctx, "smooth", 0, prec, rows, 0)
        n = nx * ny * nz
        u = ctx.to_device(W.uniform_pm1(33, 1, n), dtype=dt)
        f = ctx.to_device(W.uniform_pm1(33, 2, n), dtype=dt)
        G.line_smooth(ctx, 0, f, u, nsweeps=3)
        outs.append(ctx.from_device(u))    # the grid's elements (padding is not part of u)
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("grid", [(128, 6, 128), (64, 4, 64), (192, 2, 32)])
def test_two_wavefront_smoother_norm(grid, prec):
    """The norm-computing smoother of the multigrid solve in the two-wavefront
    form: the same iterate as the one-wavefront form, and the same
    ||f - A u||^2 up to the summation order of its workgroup partials."""
    import paper_1402_3545_amd as G
    nx, ny, nz = grid
    ctx, orc, _ = problem(nx, ny, nz, nlevels=1, seed=29)
    f = W.uniform_pm1(34, 2, nx * ny * nz)
    fd = ctx.to_device(f)
    res = []
    for rows in (2, 3):
        G.gmg_set_launch(ctx, "smooth", 0, prec, rows, 0)
        G.gmg_set_graphs(ctx, False)
        ud = ctx.empty()
        it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-300, maxit=3, check=False)
        res.append((ctx.from_device(ud), hist))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.allclose(res[0][1], res[1][1], rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec_precond", [0, 1])
def test_autotune_then_solve_matches_oracle(prec_precond):
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=prec_precond)
    f = w.rhs()
    fd = ctx.to_device(f)
    ud0 = ctx.empty()
    it0, rel0, _, st0 = G.gmg_solve(ctx, fd, ud0, rtol=1e-10, maxit=60)
    G.gmg_autotune(ctx, reps=2)
    table = G.launch_table(ctx)
    assert all(r in (1, 4, 8, 16) and 0 <= g <= 8 for k, (r, g) in table.items()
               if not k.startswith(("smooth/", "prolong_smooth/")))
    # the folded prolongation is on (2, 3) or off (4)
    assert all(r in (2, 3, 4) and 0 <= g <= 8 for k, (r, g) in table.items()
               if k.startswith("prolong_smooth/"))
    # the smoother may also take the staged-neighbour forms (rows = 2, 3)
    assert all(r in (1, 2, 3, 4) and 0 <= g <= 8 for k, (r, g) in table.items()
               if k.startswith("smooth/"))
    ud = ctx.empty()
    it, rel, _, st = G.gmg_solve(ctx, fd, ud, rtol=1e-10, maxit=60)
    assert st == st0 == 0 and it == it0
    assert rel == pytest.approx(rel0, rel=1e-6)
    u = ctx.from_device(ud)
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-10
    # the line-preconditioned CG after tuning
    ud.zero_()
    itc, relc, _, stc = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=500)
    assert stc == 0
    true_rel = orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-8


def test_launch_shape_validation():
    import paper_1402_3545_amd as G
    ctx, _, _ = problem(16, 16, 8, nlevels=2)
    G.gmg_set_launch(ctx, "spmv", 1, G.GMG_F32, 16, 3)
    assert G.gmg_get_launch(ctx, "spmv", 1, G.GMG_F32) == (16, 3)
    G.gmg_set_launch(ctx, "line_solve", 0, G.GMG_F64, 1, 0)     # cyclic reduction
    assert G.gmg_get_launch(ctx, "line_solve", 0, G.GMG_F64) == (1, 0)
    G.gmg_set_launch(ctx, "smooth", 1, G.GMG_F32, 2, 4)         # staged neighbours
    assert G.gmg_get_launch(ctx, "smooth", 1, G.GMG_F32) == (2, 4)
    G.gmg_set_launch(ctx, "smooth", 0, G.GMG_F64, 3, 0)         # two wavefronts per column
    G.gmg_set_launch(ctx, "prolong_smooth", 0, G.GMG_F64, 3, 2)
    assert G.gmg_get_launch(ctx, "prolong_smooth", 0, G.GMG_F64) == (3, 2)
    for bad in [("spmv", 2, 0, 4, 0), ("spmv", 0, 2, 4, 0), ("spmv", 0, 0, 5, 0),
                ("spmv", 0, 0, 4, -1), ("spmv", 0, 0, 4, 5000), (99, 0, 0, 4, 0),
                ("spmv", 0, 0, 1, 0), ("cg_tridiag", 0, 0, 1, 0), ("line_solve", 0, 0, 2, 0),
                ("spmv", 0, 0, 2, 0), ("line_solve", 0, 0, 3, 0), ("prolong_smooth", 0, 0, 1, 0)]:
        with pytest.raises(G.GmgError):
            G.gmg_set_launch(ctx, *bad)
    with pytest.raises(G.GmgError):
        G.gmg_autotune(ctx, reps=0)


def test_timing_filter_times_only_selected_kinds():
    """With a filter only the selected kernel kinds are bracketed by events;
    the solve itself is unchanged (bitwise)."""
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, _, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                        kh_model=w.kh_model)
    f = w.rhs()
    fd = ctx.to_device(f)
    outs = []
    for kinds in (None, ["cg_spmv"], ["smooth", "prolongate"]):
        ud = ctx.empty()
        G.gmg_timing_filter(ctx, kinds)
        G.gmg_timing_enable(ctx, True)
        G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=500)
        G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=50)
        table = G.gmg_timing_table(ctx)
        G.gmg_timing_enable(ctx, False)
        timed = {k[0] for k in table}
        if kinds is None:
            assert {"cg_spmv", "cg_tridiag", "smooth", "prolongate"} <= timed
        else:
            assert timed == set(kinds)
        outs.append(ud.clone())
    G.gmg_timing_filter(ctx, None)
    assert all(torch.equal(outs[0], o) for o in outs[1:])
