"""Failure handling on the device: non-finite input must end every solver
with GMG_ENOCONV at once (never a hang, never a reported convergence), and in
a batched solve only the affected (instance, rhs) pair fails while the others
still converge.  The non-finite values come from the inputs, so every kernel
runs its normal path and exits."""

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


def _solvers(G):
    return {
        "mg": lambda c, f, u: G.gmg_solve(c, f, u, rtol=1e-8, maxit=20, check=False),
        "pcg": lambda c, f, u: G.pcg_solve(c, f, u, rtol=1e-8, maxit=20, check=False),
        "fcg_vcycle": lambda c, f, u: G.pcg_solve(c, f, u, rtol=1e-8, maxit=20, precond=1,
                                                  check=False),
        "fcg_line": lambda c, f, u: G.pcg_solve(c, f, u, rtol=1e-8, maxit=20, precond=2,
                                                check=False),
    }


@pytest.mark.parametrize("where", ["rhs_nan", "rhs_huge", "guess_inf"])
@pytest.mark.parametrize("prec_precond", [0, 1])
def test_non_finite_input_stops_every_solver(where, prec_precond):
    import paper_1402_3545_amd as G
    nx, ny, nz = 32, 16, 8
    ctx, _, _ = problem(nx, ny, nz, nlevels=3, prec_precond=prec_precond)
    f = W.rhs(3, 0, nx, ny, nz)
    u0 = np.zeros_like(f)
    if where == "rhs_nan":
        f[777] = np.nan
    elif where == "rhs_huge":
        f[::5] = 1e300          # ||f||^2 overflows to Inf
    else:
        u0[123] = np.inf
    for name, solve in _solvers(G).items():
        fd, ud = ctx.to_device(f), ctx.to_device(u0)
        it, rel, hist, st = solve(ctx, fd, ud)
        assert st == G.GMG_ENOCONV, (name, st)
        assert it == 0, (name, it)
        assert G.gmg_last_error()
    # the context is still usable afterwards
    fd, ud = ctx.to_device(W.rhs(3, 0, nx, ny, nz)), ctx.empty()
    it, rel, _, st = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=60)
    assert st == 0 and rel < 1e-8


def test_batched_pair_with_nan_fails_alone():
    import oracle
    import paper_1402_3545_amd as G
    kws = [dict(nx=n, ny=n, nz=nz, nlevels=L, kv=1e4, sigma=1.0, zfaces=W.quadratic_faces(nz),
                kh=W.kh_uniform(6000 + q, n, n))
           for q, (n, nz, L) in enumerate([(32, 8, 3), (48, 16, 2)])]
    b = G.GmgBatch(kws, nrhs=2)
    fh, fs, us = [], [], []
    for q, kw in enumerate(kws):
        for r in range(2):
            f = W.uniform_pm1(6000 + q, 1 + r, kw["nx"] * kw["ny"] * kw["nz"])
            if (q, r) == (1, 0):
                f[5] = np.nan
            fh.append(f)
            fs.append(b.to_device(f, q))
            us.append(b.empty(q))
    it, rel, st = G.gmg_batch_solve(b, fs, us, rtol=1e-8, maxit=60, check=False)
    assert st == G.GMG_ENOCONV
    assert it[2] == 0
    for pq in (0, 1, 3):
        q = pq // 2
        kw = kws[q]
        orc = oracle.OracleProblem(kw["nx"], kw["ny"], kw["nz"], kw["nlevels"], kv=kw["kv"],
                                   sigma=1.0, zfaces=kw["zfaces"], kh=kw["kh"], matfree=True)
        u = b.from_device(us[pq], q)
        true_rel = orc.residual_norm2_rows(fh[pq], u) ** 0.5 / np.linalg.norm(fh[pq])
        assert true_rel < 1e-8, (pq, true_rel)


@pytest.mark.parametrize("precond", [1, 2])
def test_flexible_cg_breakdown_keeps_the_previous_iterate(precond):
    """Right-hand-side values of 1e39 are finite in FP64 but overflow the FP32
    copy of the residual that the FP32 preconditioner works on, so <p, Ap> of
    the first direction is not finite: the flexible CG must stop with a
    breakdown (GMG_ENOCONV, no iteration counted) and return its last iterate,
    the initial guess, bit for bit."""
    import paper_1402_3545_amd as G
    nx, ny, nz = 32, 16, 8
    ctx, _, _ = problem(nx, ny, nz, nlevels=3, prec_precond=1)
    f = W.rhs(4, 0, nx, ny, nz)
    f[::7] = 1e39
    u0 = W.rhs(4, 1, nx, ny, nz)
    fd, ud = ctx.to_device(f), ctx.to_device(u0)
    before = ud.clone()
    it, rel, hist, st = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=20, precond=precond,
                                    check=False)
    assert st == G.GMG_ENOCONV
    assert it == 0
    assert "breakdown" in G.gmg_last_error()
    assert torch.equal(ud, before)
    assert np.isfinite(rel)
