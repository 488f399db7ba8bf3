"""Device-side iteration loops and their hipGraph replays.

Every solver keeps its stopping test on the device and gates the kernels of
iterations enqueued past convergence; batches of iterations are replayed from
a captured hipGraph.  The graph path must give bitwise the results of the
same kernels launched one by one, on every replay of a cached graph (with
other work and synchronisations between the solves), after a launch-shape
change, and for single-level hierarchies (whose cycle ends in a gated copy).
The solvers' parity with the oracle is checked in test_gpu_solvers.py and
the other solver tests, which run the graph path (the default).
"""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


SOLVERS = {
    # name: (prec_precond, call)
    "mg_f64": (0, lambda G, c, f, u: G.gmg_solve(c, f, u, rtol=1e-9, maxit=60, check=False)),
    "mg_mixed": (1, lambda G, c, f, u: G.gmg_solve(c, f, u, rtol=1e-9, maxit=60, check=False)),
    "pcg_f64": (0, lambda G, c, f, u: G.pcg_solve(c, f, u, rtol=1e-9, maxit=500, check=False)),
    "fcg_vcycle": (1, lambda G, c, f, u: G.pcg_solve(c, f, u, rtol=1e-9, maxit=60, precond=1,
                                                     check=False)),
    "fcg_line": (1, lambda G, c, f, u: G.pcg_solve(c, f, u, rtol=1e-9, maxit=500, precond=2,
                                                   check=False)),
}


def _run(G, ctx, call, fd, u0):
    ud = u0.clone()
    it, rel, hist, st = call(G, ctx, fd, ud)
    torch.cuda.synchronize()
    return ud, it, rel, np.asarray(hist), st


@pytest.mark.parametrize("levels,ncoarse", [(3, 2), (1, 2), (1, 1), (1, 3)])
@pytest.mark.parametrize("name", list(SOLVERS))
def test_graph_replays_equal_direct_launches(name, levels, ncoarse):
    import paper_1402_3545_amd as G
    prec, call = SOLVERS[name]
    nx, ny, nz = 96, 64, 40
    ctx, _, _ = problem(nx, ny, nz, nlevels=levels, kv=1e3, seed=17, prec_precond=prec,
                        ncoarse=ncoarse)
    fd = ctx.to_device(W.rhs(17, 0, nx, ny, nz))
    u0 = ctx.to_device(0.1 * W.rhs(17, 1, nx, ny, nz))
    G.gmg_set_graphs(ctx, False)
    ref = _run(G, ctx, call, fd, u0)
    # a single level is block Jacobi alone: it need not reach the tolerance,
    # and a solve stopped at maxit must replay just the same
    assert ref[4] == 0 or (levels == 1 and ref[4] == G.GMG_ENOCONV), (name, G.gmg_last_error())
    G.gmg_set_graphs(ctx, True)
    # other work on the stream between the replays of the cached graph
    x = ctx.to_device(W.rhs(17, 2, nx, ny, nz))
    y = ctx.empty()
    for rep in range(3):
        got = _run(G, ctx, call, fd, u0)
        assert torch.equal(got[0], ref[0]), (name, rep)
        assert got[1] == ref[1] and got[4] == ref[4], (name, rep, got[1], ref[1])
        assert np.array_equal(got[3], ref[3]), (name, rep)
        assert got[2] == ref[2], (name, rep)
        G.spmv(ctx, 0, x, y)
        torch.cuda.synchronize()


def test_launch_shape_change_recaptures():
    import paper_1402_3545_amd as G
    nx, ny, nz = 128, 64, 32
    ctx, _, _ = problem(nx, ny, nz, nlevels=3, seed=19)
    fd = ctx.to_device(W.rhs(19, 0, nx, ny, nz))
    u0 = ctx.empty()
    call = SOLVERS["mg_f64"][1]
    first = _run(G, ctx, call, fd, u0)
    # a different smoother shape on level 1 (bitwise the same results) and a
    # different tile order for the residual-restriction
    G.gmg_set_launch(ctx, "smooth", 1, 0, 1, 0)
    G.gmg_set_launch(ctx, "residual_restrict", 0, 0, 8, 2)
    after = _run(G, ctx, call, fd, u0)
    G.gmg_set_graphs(ctx, False)
    direct = _run(G, ctx, call, fd, u0)
    assert torch.equal(after[0], direct[0])
    assert after[1] == direct[1] == first[1]
    assert np.array_equal(after[3], direct[3])


@pytest.mark.parametrize("prec", [0, 1])
def test_multigrid_reads_the_device_state_rarely(prec):
    """A multigrid solve of ~15 cycles waits for the device at most three
    times (refinement: four, its batches come in pairs); line-PCG's ~70
    iterations at most six."""
    import paper_1402_3545_amd as G
    nx, ny, nz = 256, 256, 64
    ctx, _, _ = problem(nx, ny, nz, nlevels=4, kv=1e4, seed=23, prec_precond=prec)
    fd = ctx.to_device(W.rhs(23, 0, nx, ny, nz))
    ud = ctx.empty()
    it, rel, _, st = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=60)
    polls = G.gmg_solver_polls(ctx)
    assert st == 0 and rel < 1e-8 and it >= 10, (it, rel)
    assert polls <= (3 if prec == 0 else 4), (it, polls)
    if prec == 0:
        ud.zero_()
        it, rel, _, st = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=500)
        assert st == 0 and G.gmg_solver_polls(ctx) <= 6, (it, G.gmg_solver_polls(ctx))
