"""The paper's model problem across CFL numbers (Sec. 5.2) at a size the
oracle solves in seconds: the flat box with Dirichlet side walls and Neumann
ends, K = (nu_CFL h / 2)^2, hierarchies from 3 levels down to a single
column.  Multigrid takes exactly the oracle's number of cycles with the same
residual history; CG ends within one iteration of the oracle's."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import max_rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _pair(fb, matfree=False):
    import oracle
    import paper_1402_3545_amd as G
    kw = fb.params()
    ctx = G.GmgContext(fb.n, fb.n, fb.nz, fb.nlevels, **kw)
    orc = oracle.OracleProblem(fb.n, fb.n, fb.nz, fb.nlevels, matfree=matfree, **kw)
    return ctx, orc


@pytest.mark.parametrize("L", [3, 5, 7])
@pytest.mark.parametrize("nu", [2.1, 8.4, 84.0, 840.0])
def test_mg_across_cfl_numbers(nu, L):
    import paper_1402_3545_amd as G
    fb = W.FlatBox(64, 16, nu, L)
    ctx, orc = _pair(fb)
    f = fb.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, fb.rtol, 200, check=False)
    u_ref, it_ref, hist_ref, st_ref = orc.mg_solve(f, rtol=fb.rtol, maxit=200)
    assert st == st_ref == 0 and it == it_ref
    # rounding floor of the residual norms, as for the other runs with a stiff
    # vertical coupling
    assert np.allclose(hist, hist_ref, rtol=1e-10, atol=1e-12)
    assert max_rel(ctx.from_device(ud), u_ref, np.abs(u_ref).max()) < 1e-9


@pytest.mark.parametrize("nu", [2.1, 8.4, 84.0])
def test_pcg_across_cfl_numbers(nu):
    import paper_1402_3545_amd as G
    fb = W.FlatBox(64, 16, nu, 1)
    ctx, orc = _pair(fb)
    f = fb.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, fb.rtol, 5000)
    _, it_ref, hist_ref, rt_ref, st_ref = orc.pcg_solve(f, rtol=fb.rtol, maxit=5000)
    assert st == st_ref == 0 and abs(it - it_ref) <= 1
    m = min(it, it_ref) + 1
    assert np.allclose(hist[:m], hist_ref[:m], rtol=1e-6, atol=0)
    assert orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f) \
        < 1.01 * fb.rtol


def test_sweep_size_multigrid_sampled_against_oracle():
    """At the sweep's own size (512^2 x 128, 10 levels down to one column,
    nu_CFL = 840): the solution's FP64 true residual, computed by the oracle's
    row-wise operator on every row, meets the tolerance, and the returned
    relative residual agrees with it."""
    import paper_1402_3545_amd as G
    fb = W.FlatBox(512, 128, 840.0, 10)
    ctx, orc = _pair(fb, matfree=True)
    f = fb.rhs()
    fd, ud = ctx.to_device(f), ctx.empty()
    it, rel, hist, st = G.gmg_solve(ctx, fd, ud, fb.rtol, 100)
    assert st == 0 and it < 30
    true_rel = orc.residual_norm2_rows(f, ctx.from_device(ud)) ** 0.5 / np.linalg.norm(f)
    assert true_rel < fb.rtol and true_rel == pytest.approx(rel, rel=1e-6)
