"""Full-size batched workload: 64 instances with seeded sizes n x n x n_z,
n in {128, 256, 384, 512}, n_z in {32, 64, 128}, 4 right-hand sides each
(about 2.45e9 unknown-RHS pairs in one batched context), FP32 V-cycles inside
FP64 refinement to 1e-8.  Every (instance, rhs) pair must converge; the
library's reported FP64 relative residual is checked against the oracle's FP64
true residual (matrix-free, every row) on one right-hand side of sixteen
instances, covering every size class present."""

import numpy as np
import pytest

import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")


def test_full_batched_workload():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import oracle
    import paper_1402_3545_amd as G
    insts = W.batched_instances()
    nrhs = insts[0].nrhs
    kws = [dict(nx=w.nx, ny=w.ny, nz=w.nz, nlevels=w.nlevels, kv=w.kv, sigma=w.sigma,
                zfaces=w.zfaces(), kh=w.kh()) for w in insts]
    b = G.GmgBatch(kws, nrhs=nrhs)
    # one checked pair per instance for the first sixteen instances, plus the
    # first instance of each (n, n_z) class
    first = {}
    for q, w in enumerate(insts):
        first.setdefault((w.nx, w.nz), q)
    checked = {(q, q % nrhs) for q in range(16)} | {(q, 0) for q in first.values()}
    fs, us, fh = [], [], {}
    for q, w in enumerate(insts):
        for r in range(nrhs):
            f = w.rhs(r)
            if (q, r) in checked:
                fh[(q, r)] = f
            fs.append(b.to_device(f, q))
            us.append(b.empty(q))
    it, rel, st = G.gmg_batch_solve(b, fs, us, rtol=1e-8, maxit=60)
    assert st == 0, G.gmg_last_error()
    assert (rel < 1e-8).all() and (it > 0).all() and (it < 60).all()
    for (q, r), f in sorted(fh.items()):
        w = insts[q]
        orc = oracle.OracleProblem(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma,
                                   zfaces=kws[q]["zfaces"], kh=kws[q]["kh"], matfree=True)
        u = b.from_device(us[q * nrhs + r], q)
        true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
        assert true_rel < 1e-8, (q, r, true_rel)
        assert true_rel == pytest.approx(rel[q * nrhs + r], rel=1e-5), (q, r)
    del fs, us
    b.close()
    torch.cuda.empty_cache()
