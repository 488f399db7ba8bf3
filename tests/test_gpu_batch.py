"""Batched solves (independent instances of uneven sizes, several right-hand
sides, one grouped launch per V-cycle phase, one hipGraph replay per
refinement step).  Each (instance, rhs) pair is checked against the oracle's
FP64 true residual, and against the single-instance FP32-cycle refinement,
which runs the same per-element arithmetic through the ungrouped kernels."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (n, nz, levels): uneven sizes, column heights in every compile-time class,
# coarsest levels at different depths, a single-level instance; 32 and 128
# layers alone in their class (the exact-height grouped launches), 50 beside
# 64 (one launch of the general form for both)
INSTANCES = [(32, 8, 3), (64, 16, 4), (48, 5, 2), (16, 32, 3), (40, 64, 2), (24, 3, 1),
             (64, 128, 4), (32, 50, 2)]
NRHS = 2


def _inst(q, n, nz, L):
    return dict(nx=n, ny=n, nz=nz, nlevels=L, kv=1e4, sigma=1.0,
                zfaces=W.quadratic_faces(nz), kh=W.kh_uniform(4000 + q, n, n))


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1402_3545_amd as G
    kws = [_inst(q, *s) for q, s in enumerate(INSTANCES)]
    return G.GmgBatch(kws, nrhs=NRHS), kws


def test_batched_solve_matches_oracle_and_single_solves(batch):
    import oracle
    import paper_1402_3545_amd as G
    b, kws = batch
    fs, us, fh = [], [], []
    for q, kw in enumerate(kws):
        n = kw["nx"] * kw["ny"] * kw["nz"]
        for r in range(NRHS):
            f = W.uniform_pm1(4000 + q, 1 + r, n)
            fh.append(f)
            fs.append(b.to_device(f, q))
            us.append(b.empty(q))
    it, rel, st = G.gmg_batch_solve(b, fs, us, rtol=1e-8, maxit=60)
    assert st == 0, G.gmg_last_error()
    for q, kw in enumerate(kws):
        orc = oracle.OracleProblem(kw["nx"], kw["ny"], kw["nz"], kw["nlevels"], kv=kw["kv"],
                                   sigma=1.0, zfaces=kw["zfaces"], kh=kw["kh"], matfree=True)
        ctx = G.GmgContext(prec_precond=G.GMG_F32, **kw)
        for r in range(NRHS):
            pq = q * NRHS + r
            u = b.from_device(us[pq], q)
            true_rel = orc.residual_norm2_rows(fh[pq], u) ** 0.5 / np.linalg.norm(fh[pq])
            assert true_rel < 1e-8, (q, r, true_rel)
            assert true_rel == pytest.approx(rel[pq], rel=1e-5)
            # the single-instance refinement runs the same arithmetic
            ud = ctx.empty()
            it1, rel1, _, st1 = G.gmg_solve(ctx, ctx.to_device(fh[pq]), ud, rtol=1e-8, maxit=60)
            assert st1 == 0 and it1 == it[pq], (q, r, it1, it[pq])
            u1 = ctx.from_device(ud)
            assert np.abs(u1 - u).max() <= 1e-12 * np.abs(u1).max()


def test_batched_solve_twice_and_zero_rhs(batch):
    """Graph replays leave no state behind: a second solve gives the same
    result; a zero right-hand side converges at once."""
    import paper_1402_3545_amd as G
    b, kws = batch
    fs, us = [], []
    for q, kw in enumerate(kws):
        n = kw["nx"] * kw["ny"] * kw["nz"]
        for r in range(NRHS):
            f = W.uniform_pm1(77 + q, 1 + r, n) if (q + r) % 3 else np.zeros(n)
            fs.append(b.to_device(f, q))
            us.append(b.empty(q))
    it1, rel1, st1 = G.gmg_batch_solve(b, fs, us, rtol=1e-8, maxit=60)
    sol1 = [u.clone() for u in us]
    for u in us:
        u.zero_()
    it2, rel2, st2 = G.gmg_batch_solve(b, fs, us, rtol=1e-8, maxit=60)
    assert st1 == 0 and st2 == 0
    assert np.array_equal(it1, it2)
    for a, c in zip(sol1, us):
        assert torch.equal(a, c)
    for q in range(len(kws)):
        for r in range(NRHS):
            if (q + r) % 3 == 0:
                assert it1[q * NRHS + r] == 0


def test_batched_maxit_reports_noconv(batch):
    import paper_1402_3545_amd as G
    b, kws = batch
    fs = [b.to_device(W.uniform_pm1(5, 1, kw["nx"] * kw["ny"] * kw["nz"]), q)
          for q, kw in enumerate(kws) for _ in range(NRHS)]
    us = [b.empty(q) for q, kw in enumerate(kws) for _ in range(NRHS)]
    it, rel, st = G.gmg_batch_solve(b, fs, us, rtol=1e-8, maxit=2, check=False)
    assert st == G.GMG_ENOCONV
    assert (it == 2).all()
