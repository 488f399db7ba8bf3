"""Parity of the V-cycle and of the MG / CG / mixed-precision solvers with the
CPU oracle on seeded synthetic inputs.

Bars: the V-cycle is a fixed linear map; FP64 cycles agree with the oracle to
1e-11 of max|u| (a few kernels' worth of 1e-15-level differences).  FP64 MG
takes exactly the oracle's number of cycles with residual histories within
1e-10 relative; FP64 CG ends within one iteration of the oracle and meets the
tolerance in the true residual.  Mixed precision (FP32 cycles inside FP64
refinement) is judged by the true FP64 relative residual, computed by the
oracle from the returned solution; its error against the oracle's FP64
solution is recorded, not gated beyond that."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import max_rel, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


VC = [((4, 4, 8), 1, 2), ((8, 8, 4), 2, 2), ((8, 8, 3), 3, 3), ((64, 64, 64), 4, 2),
      ((40, 24, 37), 3, 2), ((32, 64, 128), 5, 2),
      # full 64-column tiles on the fine and coarse levels (the fused
      # residual-restriction passes neighbours by lane shifts there), and
      # full tiles beside a ragged one
      ((256, 4, 33), 3, 2), ((264, 6, 40), 2, 2)]


@pytest.mark.parametrize("shape,L,nc", VC)
def test_vcycle_f64(shape, L, nc):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, nlevels=L, ncoarse=nc, seed=10)
    n = nx * ny * nz
    f = W.uniform_pm1(10, 1, n)
    u = W.uniform_pm1(10, 2, n)
    fd, ud = ctx.to_device(f), ctx.to_device(u)
    G.gmg_vcycle(ctx, fd, ud)
    ref = orc.vcycle(f, u)
    assert max_rel(ctx.from_device(ud), ref, np.abs(ref).max()) < 1e-11


@pytest.mark.parametrize("shape,L,nc", VC)
def test_vcycle_f32(shape, L, nc):
    import paper_1402_3545_amd as G
    nx, ny, nz = shape
    ctx, orc, _ = problem(nx, ny, nz, nlevels=L, ncoarse=nc, seed=10, prec_precond=1)
    n = nx * ny * nz
    f = W.uniform_pm1(10, 1, n).astype(np.float32).astype(np.float64)
    u = W.uniform_pm1(10, 2, n).astype(np.float32).astype(np.float64)
    fd, ud = ctx.to_device(f, dtype=torch.float32), ctx.to_device(u, dtype=torch.float32)
    G.gmg_vcycle(ctx, fd, ud)
    ref = orc.vcycle(f, u)
    assert max_rel(ctx.from_device(ud), ref, np.abs(ref).max()) < 1e-4


def _small():
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model)
    return w, ctx, orc


def test_mg_solve_matches_oracle_history():
    import paper_1402_3545_amd as G
    w, ctx, orc = _small()
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=w.rtol, maxit=50)
    u_ref, it_ref, hist_ref, st_ref = orc.mg_solve(f, rtol=w.rtol, maxit=50)
    assert st == 0 and st_ref == 0
    assert it == it_ref
    assert np.allclose(hist, hist_ref, rtol=1e-10, atol=0)
    u = ctx.from_device(ud)
    assert max_rel(u, u_ref, np.abs(u_ref).max()) < 1e-10
    assert orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f) < w.rtol


def test_mg_solve_tight_tolerance():
    import paper_1402_3545_amd as G
    w, ctx, orc = _small()
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-10, maxit=100)
    _, it_ref, _, _ = orc.mg_solve(f, rtol=1e-10, maxit=100)
    assert st == 0 and it == it_ref
    assert (np.diff(hist) < 0).all()
    u = ctx.from_device(ud)
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-10 and true_rel == pytest.approx(rel, rel=1e-6)


def test_pcg_line_matches_oracle():
    import paper_1402_3545_amd as G
    w, ctx, orc = _small()
    f = w.rhs()
    for rtol in (w.rtol, 1e-8):
        fd, ud = ctx.to_device(f), ctx.empty()
        it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=rtol, maxit=500)
        u_ref, it_ref, hist_ref, rt_ref, st_ref = orc.pcg_solve(f, rtol=rtol, maxit=500)
        assert st == 0 and st_ref == 0
        assert abs(it - it_ref) <= 1
        m = min(it, it_ref) + 1
        assert np.allclose(hist[:m], hist_ref[:m], rtol=1e-6, atol=0)
        u = ctx.from_device(ud)
        true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
        assert true_rel < rtol * 1.01
        assert true_rel == pytest.approx(rel, rel=1e-6)


@pytest.mark.parametrize("grid", ["small", "wide"])
def test_mixed_precision_refinement_reaches_fp64_tolerance(grid):
    import paper_1402_3545_amd as G
    w = W.SMALL
    if grid == "wide":
        # full 64-column tiles beside a ragged one in the FP64 update +
        # residual (east/west of u + e by lane shifts)
        w = W.Workload("wide-200x8x40", 200, 8, 40, 3, 1e5, 1.0, 6, "uniform", 1e-8)
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=1)
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=60)
    _, it64, _, _ = orc.mg_solve(f, rtol=1e-8, maxit=60)
    assert st == 0
    u = ctx.from_device(ud)
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-8
    assert it <= it64 + 2          # FP32 cycles cost at most a couple of extra cycles
    u_ref, _, _, _ = orc.mg_solve(f, rtol=1e-12, maxit=100)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    assert err < 1e-6, err


def test_solvers_degenerate_cases():
    import paper_1402_3545_amd as G
    ctx, orc, _ = problem(8, 8, 4, nlevels=2)
    fd, ud = ctx.empty(), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=10)   # f = 0
    assert st == 0 and it == 0 and rel == 0.0
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=10)
    assert st == 0 and it == 0
    f = W.uniform_pm1(1, 1, 8 * 8 * 4)
    fd = ctx.to_device(f)
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=0, check=False)
    assert st == G.GMG_ENOCONV and it == 0
    it, rel, hist, st = G.pcg_solve(ctx, fd, ctx.empty(), rtol=1e-30, maxit=3, check=False)
    assert st == G.GMG_ENOCONV and it == 3
    with pytest.raises(G.GmgError):
        G.gmg_solve(ctx, fd, ud, rtol=0.0)
    with pytest.raises(G.GmgError):
        G.pcg_solve(ctx, fd, ud, rtol=1e-8, precond=3)


@pytest.mark.parametrize("prec_precond", [0, 1])
def test_flexible_cg_with_multigrid_preconditioner(prec_precond):
    """Flexible CG with one V-cycle (FP64 or FP32) per iteration.  The oracle has
    no flexible CG; the result is judged by the FP64 true residual the oracle
    computes from the returned solution and by its distance to the oracle's
    tightly converged FP64 multigrid solution."""
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=prec_precond)
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=60, precond=1)
    _, it_mg, _, _ = orc.mg_solve(f, rtol=1e-8, maxit=60)
    assert st == 0
    assert it <= it_mg                 # a Krylov wrapper never needs more cycles than plain MG
    u = ctx.from_device(ud)
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-8
    assert true_rel == pytest.approx(rel, rel=1e-6)
    u_ref, _, _, _ = orc.mg_solve(f, rtol=1e-12, maxit=100)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-6


@pytest.mark.parametrize("prec_precond", [0, 1])
def test_flexible_cg_with_line_preconditioner(prec_precond):
    """Flexible CG with the line preconditioner alone (precond = 2).  In FP64
    it is PCG up to rounding: within one iteration of the oracle's PCG.  With
    the FP32 line solve (an inexact preconditioner, relative error ~1e-6 per
    application) the flexible recurrence still reaches the FP64 tolerance in
    the true residual, with at most a few more iterations."""
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=prec_precond)
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=500, precond=2)
    u_ref, it_ref, _, _, st_ref = orc.pcg_solve(f, rtol=1e-8, maxit=500)
    assert st == 0 and st_ref == 0
    if prec_precond == 0:
        assert abs(it - it_ref) <= 1
    else:
        assert it_ref - 1 <= it <= it_ref + 4
    u = ctx.from_device(ud)
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-8 and true_rel == pytest.approx(rel, rel=1e-6)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-6


def test_mg_with_cyclic_reduction_on_coarse_levels():
    """The V-cycle with the coarse-level line kernels switched to one
    wavefront per column follows the oracle's history."""
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model)
    for lvl in range(1, ctx.nlevels):
        G.gmg_set_launch(ctx, "line_solve", lvl, G.GMG_F64, 1, 0)
        G.gmg_set_launch(ctx, "smooth", lvl, G.GMG_F64, 1, 0)
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=w.rtol, maxit=50)
    u_ref, it_ref, hist_ref, st_ref = orc.mg_solve(f, rtol=w.rtol, maxit=50)
    assert st == 0 and it == it_ref
    assert np.allclose(hist, hist_ref[:len(hist)], rtol=1e-10, atol=0)


@pytest.mark.parametrize("prec_precond", [0, 1])
def test_mg_with_staged_smoother_on_every_level(prec_precond):
    """The V-cycle with the smoother's neighbours staged in LDS on every level
    (the norm-computing pre-smoothing step included): FP64 follows the oracle's
    history; the FP32-cycle refinement reaches the FP64 tolerance."""
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=prec_precond)
    for lvl in range(ctx.nlevels):
        for p in (G.GMG_F64, G.GMG_F32):
            G.gmg_set_launch(ctx, "smooth", lvl, p, 2, 0)
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=50)
    u_ref, it_ref, hist_ref, st_ref = orc.mg_solve(f, rtol=1e-8, maxit=50)
    assert st == 0
    if prec_precond == 0:
        assert it == it_ref
        # to 1e-8 the last entries sit near the residual's rounding floor
        assert np.allclose(hist, hist_ref[:len(hist)], rtol=1e-10, atol=1e-14)
    else:
        assert it <= it_ref + 2
    u = ctx.from_device(ud)
    assert orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f) < 1e-8


@pytest.mark.parametrize("precond", [1, 2])
@pytest.mark.parametrize("maxit", [1, 2, 5])
def test_flexible_cg_stopped_early_returns_its_last_iterate(precond, maxit):
    """The flexible CG applies each step's u += alpha p one kernel later (and
    the last one after the loop): stopped after `maxit` iterations, the
    returned u must be the maxit-th iterate, whose true residual equals the
    recursively updated one of the same iteration."""
    import paper_1402_3545_amd as G
    w, ctx, orc = _small()
    f = w.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=1e-14, maxit=maxit, precond=precond,
                                    check=False)
    assert st == G.GMG_ENOCONV and it == maxit
    true_rel = orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f)
    assert true_rel == pytest.approx(hist[maxit], rel=1e-6)
    assert true_rel == pytest.approx(rel, rel=1e-9)
