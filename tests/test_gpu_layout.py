"""Layout conversion (z-contiguous host order <-> x-contiguous device order)
and solves from host memory.

The conversion is a permutation, so it must be bit-exact against the plain
index definition (numpy's canonical_to_xcontig in the binding) and leave the
padding columns of the x-contiguous field alone; a round trip returns the
input.  A solve from host arrays runs the same kernels on the same values as
the device-resident solve, so its solution must be bitwise identical."""

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(40, 6, 37, 1), (96, 32, 2, 2), (1024, 8, 128, 3), (33, 64, 64, 1), (64, 64, 33, 3)]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_transpose_is_the_layout_permutation(shape, dtype):
    import paper_1402_3545_amd as G
    nx, ny, nz, L = shape
    ctx, _, _ = problem(nx, ny, nz, nlevels=L)
    dt = torch.float64 if dtype == "f64" else torch.float32
    for lvl in range(L):
        cnx, cny, cnz = ctx.shape(lvl)
        ldx, elems = ctx.layout(lvl)
        z = W.uniform_pm1(50 + lvl, 1, cnx * cny * cnz)
        if dtype == "f32":
            z = z.astype(np.float32).astype(np.float64)
        zd = torch.from_numpy(z).to(dt).cuda()
        xd = torch.full((elems,), 7.0, dtype=dt, device="cuda")
        G.gmg_transpose_in(ctx, lvl, zd, xd)
        ref = G.canonical_to_xcontig(z, cnx, cny, cnz, ldx)
        got = xd.double().cpu().numpy()
        valid = np.zeros(elems, dtype=bool)
        valid.reshape(cny, cnz, ldx)[:, :, :cnx] = True
        assert np.array_equal(got[valid], ref[valid])
        assert (got[~valid] == 7.0).all()          # padding untouched
        back = torch.zeros_like(zd)
        G.gmg_transpose_out(ctx, lvl, xd, back)
        assert torch.equal(back, zd)


@pytest.mark.parametrize("method,prec_precond", [("mg", 0), ("pcg", 0), ("mg", 1), ("fcg", 1)])
def test_host_solve_equals_device_solve(method, prec_precond):
    import paper_1402_3545_amd as G
    w = W.SMALL
    ctx, orc, _ = problem(w.nx, w.ny, w.nz, nlevels=w.nlevels, kv=w.kv, seed=w.seed,
                          kh_model=w.kh_model, prec_precond=prec_precond)
    f = w.rhs()
    u = np.zeros_like(f)
    it, rel, tm, st = G.gmg_solve_host(ctx, f, u, method=method, rtol=1e-8, maxit=500)
    assert st == 0
    assert all(np.isfinite(v) and v >= 0.0 for v in tm.values())
    fd, ud = ctx.to_device(f), ctx.empty()
    if method == "mg":
        it2, rel2, _, st2 = G.gmg_solve(ctx, fd, ud, rtol=1e-8, maxit=500)
    else:
        it2, rel2, _, st2 = G.pcg_solve(ctx, fd, ud, rtol=1e-8, maxit=500,
                                        precond=0 if method == "pcg" else 1)
    assert st2 == 0 and it == it2 and rel == rel2
    assert np.array_equal(u, ctx.from_device(ud))
    true_rel = orc.residual_norm2_rows(f, u) ** 0.5 / np.linalg.norm(f)
    assert true_rel < 1e-8
    # a second call reuses the context's host-solve buffers and gives the same
    # result
    u2 = np.zeros_like(f)
    it3, rel3, _, st3 = G.gmg_solve_host(ctx, f, u2, method=method, rtol=1e-8, maxit=500)
    assert st3 == 0 and it3 == it and np.array_equal(u2, u)


def test_host_solve_in_several_staging_chunks():
    """388 MiB per field: three full 128 MiB staging chunks and a ragged
    tail, with both pinned buffers reused, for the right-hand side, the
    initial guess and the solution; the iterate after two V-cycles must be
    bitwise that of the device-resident solve from the same guess."""
    import paper_1402_3545_amd as G
    nx, ny, nz = 512, 776, 128
    kh = W.kh_uniform(29, nx, ny)
    ctx = G.GmgContext(nx, ny, nz, 3, kv=1e3, sigma=1.0, zfaces=W.quadratic_faces(nz), kh=kh)
    f = W.rhs(29, 0, nx, ny, nz)
    u0 = W.rhs(29, 1, nx, ny, nz)
    u = u0.copy()
    it, rel, tm, st = G.gmg_solve_host(ctx, f, u, method="mg", rtol=1e-14, maxit=2)
    assert st == G.GMG_ENOCONV and it == 2
    assert all(np.isfinite(v) and v >= 0.0 for v in tm.values())
    fd, ud = ctx.to_device(f), ctx.to_device(u0)
    it2, rel2, _, st2 = G.gmg_solve(ctx, fd, ud, rtol=1e-14, maxit=2, check=False)
    assert st2 == st and it2 == it and rel2 == rel
    assert np.array_equal(u, ctx.from_device(ud))


def test_host_solve_validation():
    import paper_1402_3545_amd as G
    ctx, _, _ = problem(16, 16, 8, nlevels=2)
    f = np.zeros(16 * 16 * 8)
    with pytest.raises(ValueError):
        G.gmg_solve_host(ctx, f, np.zeros(10))
    with pytest.raises(G.GmgError):
        G.gmg_solve_host(ctx, f, np.zeros_like(f), method=5)
    x = ctx.empty()
    with pytest.raises(ValueError):
        G.gmg_transpose_in(ctx, 0, x, x)
    assert G._lib.gmg_transpose_in(ctx.handle, 0, G.GMG_F64, x.data_ptr(), x.data_ptr(),
                                   None) == G.GMG_EINVAL
