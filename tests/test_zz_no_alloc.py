"""The allocation-free residual (gmg_residual_noalloc) against gmg_residual.

Both run the same residual kernel with the same launch shape and reduce the
same per-workgroup partials in the same fixed order, so r and ||r||^2 must be
bitwise equal; the only difference is where the partials live (a static
per-GPU array instead of the context's scratch) and that the norm stays on
the device.  Two calls in a row, the second on a smaller input, check that
what the first call left in the shared array is never read.  gmg_residual
itself is checked against the oracle in test_gpu_kernels.py.
"""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import abs_matvec, max_rel, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _dtype(prec):
    return torch.float64 if prec == 0 else torch.float32


def _pair(ctx, level, prec, seed):
    import paper_1402_3545_amd as G
    nx, ny, nz = ctx.shape(level)
    n = nx * ny * nz
    u = W.uniform_pm1(seed, 1, n)
    f = W.uniform_pm1(seed, 2, n)
    ud = ctx.to_device(u, level=level, dtype=_dtype(prec))
    fd = ctx.to_device(f, level=level, dtype=_dtype(prec))
    r_ref = ctx.empty(level, dtype=_dtype(prec))
    n_ref = G.gmg_residual(ctx, level, fd, ud, r_ref, norm=True)
    r = torch.full_like(r_ref, float("nan"))
    nd = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    G.gmg_residual_noalloc(ctx, level, fd, ud, r, nd)
    torch.cuda.synchronize()
    return u, f, r_ref, n_ref, r, float(nd.item())


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_residual_equals_gmg_residual(prec):
    """Level 0 of a ragged 3-level grid, then level 1 of it, then a much
    smaller grid: each bitwise equal to gmg_residual, r and norm."""
    ctx, orc, _ = problem(132, 68, 45, nlevels=3, seed=5)
    small, _, _ = problem(6, 4, 3, seed=6)
    for c, level, seed in ((ctx, 0, 21), (ctx, 1, 22), (small, 0, 23)):
        u, f, r_ref, n_ref, r, n = _pair(c, level, prec, seed)
        got, want = c.from_device(r, level), c.from_device(r_ref, level)
        assert np.array_equal(got, want), (level, prec)
        assert n == n_ref, (level, prec, n, n_ref)
        assert np.isfinite(n) and n > 0.0
    # and the first grid's level 0 against the oracle (same bar as gmg_residual)
    if prec == 0:
        u, f, _, _, r, n = _pair(ctx, 0, 0, 31)
        ref = f - orc.spmv(u)
        got = ctx.from_device(r)
        assert max_rel(got, ref, abs_matvec(orc, u) + np.abs(f)) < 1e-12
        assert abs(n - float(ref @ ref)) < 1e-12 * float(ref @ ref)


def test_noalloc_residual_without_norm():
    import paper_1402_3545_amd as G
    ctx, _, _ = problem(40, 6, 37, seed=7)
    n = 40 * 6 * 37
    ud = ctx.to_device(W.uniform_pm1(8, 1, n))
    fd = ctx.to_device(W.uniform_pm1(8, 2, n))
    r_ref, r = ctx.empty(), ctx.empty()
    G.gmg_residual(ctx, 0, fd, ud, r_ref)
    G.gmg_residual_noalloc(ctx, 0, fd, ud, r)
    torch.cuda.synchronize()
    assert np.array_equal(ctx.from_device(r), ctx.from_device(r_ref))


def test_noalloc_residual_rejects_levels_beyond_the_scratch():
    """A level needing 131073 residual workgroups (2 x 524292 columns, 2
    layers) is refused before any launch; without a norm it runs."""
    import paper_1402_3545_amd as G
    ctx = G.GmgContext(2, 524292, 2, 1, kv=1.0)
    ud, fd, r = ctx.empty(), ctx.empty(), ctx.empty()
    nd = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GmgError) as ei:
        G.gmg_residual_noalloc(ctx, 0, fd, ud, r, nd)
    assert "static scratch" in str(ei.value)
    G.gmg_residual_noalloc(ctx, 0, fd, ud, r)
    torch.cuda.synchronize()
    assert float(r.abs().max()) == 0.0
    ctx.close()
