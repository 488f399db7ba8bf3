"""Pins of the oracle's horizontal Dirichlet boundaries (bc_h = 1).

Sec. 2.1.1 takes homogeneous Dirichlet conditions on the side walls of the
horizontal domain.  In a cell-centred finite-volume scheme the wall lies half a
cell from the centre of the outermost column, so its face couples that column
to the zero boundary value with twice the interior coupling of a uniform
medium.  These tests check that reading against facts that do not come from
the oracle: the exact eigenvectors of the flat-box operator (sine modes in the
horizontal, sine or cosine modes in the vertical), second-order convergence to
manufactured solutions that vanish on the walls (also across a coefficient
jump), the flux of a constant field through the walls, exactness of the
prolongation on functions that are linear and vanish on a wall, and direct
solves and dense compositions for the solvers.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _canon(nx, ny, nz):
    return lambda i, j, k: (j * nx + i) * nz + k


def _block_diag_part(A, nz):
    blk = np.arange(A.shape[0]) // nz
    return np.where(blk[:, None] == blk[None, :], A, 0.0)


def _sine_modes(n):
    """Columns m = 1..n: sin(m pi (i + 1/2) / n) and 4 sin^2(m pi / (2n)), the
    eigenpairs of the cell-centred second difference with odd reflection at both
    ends."""
    i = np.arange(n) + 0.5
    m = np.arange(1, n + 1)
    return np.sin(np.pi * np.outer(i, m) / n), 4 * np.sin(np.pi * m / (2 * n)) ** 2


def _cosine_modes(n):
    """Columns q = 0..n-1: cos(q pi (k + 1/2) / n) and 4 sin^2(q pi / (2n)), the
    eigenpairs with even reflection (zero flux) at both ends."""
    k = np.arange(n) + 0.5
    q = np.arange(n)
    return np.cos(np.pi * np.outer(k, q) / n), 4 * np.sin(np.pi * q / (2 * n)) ** 2


@pytest.mark.parametrize("bc_v", [0, 1])
@pytest.mark.parametrize("shape", [(6, 4, 5), (2, 3, 2), (8, 8, 4)])
def test_flat_box_eigenmodes_with_walls(shape, bc_v):
    """Constant K, K_v, equidistant layers: every tensor product of horizontal
    sine modes and vertical sine (Dirichlet ends) or cosine (Neumann ends) modes
    is an eigenvector, with eigenvalue
      cell volume * (sigma + K (mu_x/hx^2 + mu_y/hy^2) + K_v mu_z/hz^2).
    The modes are a complete orthogonal basis, so this fixes the whole matrix."""
    nx, ny, nz = shape
    K, Kv, sig = 0.31, 2.7, 1.4
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=Kv, sigma=sig, zfaces=W.uniform_faces(nz),
                             kh=np.full(nx * ny, K), bc_v=bc_v, bc_h=1)
    A = p.scipy().toarray()
    hx, hy, hz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    vol = hx * hy * hz
    Vx, mx = _sine_modes(nx)
    Vy, my = _sine_modes(ny)
    Vz, mz = _sine_modes(nz) if bc_v == 0 else _cosine_modes(nz)
    scale = np.abs(A).max()
    lams = []
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                # canonical order (j*nx + i)*nz + k
                v = np.einsum("j,i,k->jik", Vy[:, b], Vx[:, a], Vz[:, c]).reshape(-1)
                lam = vol * (sig + K * (mx[a] / hx**2 + my[b] / hy**2) + Kv * mz[c] / hz**2)
                assert np.abs(A @ v - lam * v).max() < 1e-12 * scale * np.abs(v).max()
                lams.append(lam)
    ev = np.linalg.eigvalsh(A)
    assert np.allclose(np.sort(ev), np.sort(lams), rtol=1e-11, atol=0)


def _check_flat_box_modes(A, nx, ny, nz, K, Kv, sig, bc_v):
    hx, hy, hz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    vol = hx * hy * hz
    Vx, mx = _sine_modes(nx)
    Vy, my = _sine_modes(ny)
    Vz, mz = _sine_modes(nz) if bc_v == 0 else _cosine_modes(nz)
    scale = np.abs(A).max()
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                v = np.einsum("j,i,k->jik", Vy[:, b], Vx[:, a], Vz[:, c]).reshape(-1)
                lam = vol * (sig + K * (mx[a] / hx**2 + my[b] / hy**2) + Kv * mz[c] / hz**2)
                assert np.abs(A @ v - lam * v).max() < 1e-12 * scale * np.abs(v).max()


@pytest.mark.parametrize("bc_v", [0, 1])
def test_coarse_levels_are_flat_boxes_down_to_one_column(bc_v):
    """With constant K every coarse level is the flat box rediscretised on its
    own grid (coarse K = mean of the children = K), down to a single column,
    where each wall lies half a cell away on all four sides (mu = 4 per
    direction at n = 1)."""
    nx, ny, nz, L = 8, 4, 3, 3
    K, Kv, sig = 0.45, 1.3, 0.9
    p = oracle.OracleProblem(nx, ny, nz, L, kv=Kv, sigma=sig, zfaces=W.uniform_faces(nz),
                             kh=np.full(nx * ny, K), bc_v=bc_v, bc_h=1)
    for d in range(L):
        cx, cy, _ = p.shape(d)
        _check_flat_box_modes(p.scipy(d).toarray(), cx, cy, nz, K, Kv, sig, bc_v)
    assert p.shape(L - 1)[:2] == (2, 1)


def test_constant_field_flux_through_the_walls():
    """Neumann ends.  For u = 1 every interior face carries no flux; a wall face carries
    K_c (1 - 0) / (h/2) times its area, h_y dz for an x-wall and h_x dz for a
    y-wall.  So (A 1)_row = |T| sigma dz_k + dz_k (2 K_c)(n_x-walls hy/hx +
    n_y-walls hx/hy), with K_c the column's own coefficient (no neighbour across
    a wall)."""
    nx, ny, nz = 5, 4, 6
    kh = 0.2 + 3.0 * W.uniform01(21, 0, nx * ny)
    zf = W.quadratic_faces(nz)
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=40.0, sigma=0.7, zfaces=zf, kh=kh, bc_h=1,
                             bc_v=1)
    dz = np.diff(zf)
    hx, hy = 1.0 / nx, 1.0 / ny
    y = p.spmv(np.ones(nx * ny * nz)).reshape(ny, nx, nz)
    Kc = kh.reshape(ny, nx)
    nwx = (np.arange(nx) == 0).astype(float) + (np.arange(nx) == nx - 1)
    nwy = (np.arange(ny) == 0).astype(float) + (np.arange(ny) == ny - 1)
    wallflux = 2 * Kc * (nwx[None, :] * hy / hx + nwy[:, None] * hx / hy)
    expect = hx * hy * 0.7 * dz[None, None, :] + wallflux[:, :, None] * dz[None, None, :]
    scale = 40.0 * hx * hy / dz.min()
    assert np.allclose(y, expect, rtol=0, atol=1e-13 * scale)
    assert np.allclose(p.walls().reshape(ny, nx), wallflux, rtol=1e-14, atol=0)


@pytest.mark.parametrize("shape", [(4, 4, 8), (2, 6, 3), (2, 2, 4), (6, 2, 2)])
def test_walls_symmetric_m_matrix_no_wrap(shape):
    nx, ny, nz = shape
    kh = 0.5 + 1.5 * W.uniform01(11, 0, nx * ny)
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=1e3, sigma=1.0, kh=kh, bc_h=1)
    A = p.scipy().toarray()
    assert np.array_equal(A, A.T)
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all() and (np.diag(A) > 0).all()
    assert (A.sum(axis=1) > 0).all()
    np.linalg.cholesky(A)
    idx = _canon(nx, ny, nz)
    if nx > 2:
        for j in range(ny):
            for k in range(nz):
                assert A[idx(0, j, k), idx(nx - 1, j, k)] == 0.0
    if ny > 2:
        for i in range(nx):
            for k in range(nz):
                assert A[idx(i, 0, k), idx(i, ny - 1, k)] == 0.0


def test_manufactured_solution_with_walls():
    """u* = sin(pi x) sin(2 pi y) cos(pi z) vanishes on the side walls and has
    zero normal derivative at z = 0, 1; it solves -K Lap u - K_v u_zz + sigma u = g
    with g = (5 pi^2 K + pi^2 K_v + sigma) u*.  On the graded grid with Neumann
    ends the max-norm error falls at second order."""
    K, Kv, sig = 1.0, 1.0, 1.0
    errs = []
    for n in (8, 16, 32):
        nz = n
        zf = W.quadratic_faces(nz)
        p = oracle.OracleProblem(n, n, nz, 1, kv=Kv, sigma=sig, zfaces=zf, bc_v=1, bc_h=1)
        xc = (np.arange(n) + 0.5) / n
        zc = 0.5 * (zf[:-1] + zf[1:])
        X, Y, Z = xc[None, :, None], xc[:, None, None], zc[None, None, :]
        ustar = np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.cos(np.pi * Z)
        g = (5 * np.pi**2 * K + np.pi**2 * Kv + sig) * ustar
        b = (g * np.diff(zf)[None, None, :] / (n * n)).reshape(-1)
        u = spla.spsolve(p.scipy().tocsc(), b)
        errs.append(np.abs(u - ustar.reshape(-1)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 1.85 and min(orders) > 1.6, (errs, orders)


def test_manufactured_solution_with_walls_and_jump():
    """K = K1 on x < 1/2 and K2 on x > 1/2, so the walls at x = 0 and 1 lie in
    different media.  u* = sin(2 pi x)/K(x) sin(pi y) sin(pi z) vanishes on all
    four walls, is continuous with continuous flux K u_x, and solves the equation
    with g = (5 pi^2 sin(2 pi x) + (pi^2 K_v + sigma) sin(2 pi x)/K) sin(pi y) sin(pi z).
    Only a wall coupling built from the outermost column's own K keeps the
    horizontal error second order."""
    K1, K2, Kv, sig = 1.0, 10.0, 1.0, 1.0
    errs = []
    for n in (8, 16, 32):
        nz = 8
        zf = W.uniform_faces(nz)
        xc = (np.arange(n) + 0.5) / n
        Kx = np.where(xc < 0.5, K1, K2)
        p = oracle.OracleProblem(n, n, nz, 1, kv=Kv, sigma=sig, zfaces=zf,
                                 kh=np.tile(Kx, n), bc_h=1)
        zc = 0.5 * (zf[:-1] + zf[1:])
        sx, sy, sz = np.sin(2 * np.pi * xc), np.sin(np.pi * xc), np.sin(np.pi * zc)
        ustar = (sx / Kx)[None, :, None] * sy[:, None, None] * sz[None, None, :]
        # -(K u_x)_x = 4 pi^2 sin(2 pi x) sy sz; -K u_yy = pi^2 sin(2 pi x) sy sz
        gx = 4 * np.pi**2 * sx + np.pi**2 * sx + (np.pi**2 * Kv + sig) * sx / Kx
        g = gx[None, :, None] * sy[:, None, None] * sz[None, None, :]
        b = (g * np.diff(zf)[None, None, :] / (n * n)).reshape(-1)
        errs.append(spla.spsolve(p.scipy().tocsc(), b).reshape(n, n, nz))
    d1 = np.abs(errs[0] - 0.25 * sum(errs[1][b::2, a::2] for a in (0, 1) for b in (0, 1))).max()
    d2 = np.abs(errs[1] - 0.25 * sum(errs[2][b::2, a::2] for a in (0, 1) for b in (0, 1))).max()
    assert math.log2(d1 / d2) > 1.7, (d1, d2)


def test_prolongation_exact_on_functions_vanishing_on_a_wall():
    """Bilinear interpolation with odd reflection at a wall is exact for a
    bilinear function that vanishes on that wall, at every fine cell whose
    coarse stencil stays inside or reflects only across walls where the function
    vanishes."""
    nx, ny, nz = 16, 12, 2
    p = oracle.OracleProblem(nx, ny, nz, 2, bc_h=1)
    ncx, ncy = nx // 2, ny // 2
    Xc, Yc = (np.arange(ncx) + 0.5) / ncx, (np.arange(ncy) + 0.5) / ncy
    xf, yf = (np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / ny
    cases = [  # function, fine i range, fine j range where it must be exact
        (lambda x, y: x * y * 1.7, slice(0, nx - 1), slice(0, ny - 1)),
        (lambda x, y: (1 - x) * (1 - y) * 0.9, slice(1, nx), slice(1, ny)),
        (lambda x, y: x * (1 - y) * 2.1, slice(0, nx - 1), slice(1, ny)),
        (lambda x, y: (1 - x) * (0.3 + y), slice(1, nx), slice(1, ny - 1)),
    ]
    for f, si, sj in cases:
        uc = np.repeat(f(Xc[None, :], Yc[:, None])[:, :, None], nz, axis=2).reshape(-1)
        uf = p.prolongate_add(uc, np.zeros(nx * ny * nz)).reshape(ny, nx, nz)
        ref = f(xf[None, :], yf[:, None])
        for k in range(nz):
            assert np.allclose(uf[sj, si, k], ref[sj, si], rtol=0, atol=1e-14)
    # periodic wrap is gone: a delta in coarse column 0 reaches no fine column
    # on the far side
    e = np.zeros(ncx * ncy * nz)
    e[0] = 1.0
    uf = p.prolongate_add(e, np.zeros(nx * ny * nz)).reshape(ny, nx, nz)
    assert (uf[:, nx - 1] == 0).all() and (uf[ny - 1, :] == 0).all()
    assert uf[0, 0, 0] == pytest.approx((9 - 3 - 3 + 1) / 16.0, abs=0)


def _approx_inverse(p, d, rho, ncoarse):
    """Matrix of the cycle started on level d from a zero guess (Algorithm 1)."""
    A = p.scipy(d).toarray()
    Minv = np.linalg.inv(_block_diag_part(A, p.nz))
    I = np.eye(A.shape[0])
    X = rho * Minv
    if d == p.nlevels - 1:
        for _ in range(ncoarse - 1):
            X = X + rho * Minv @ (I - A @ X)
        return X
    nf, nc = p.size(d), p.size(d + 1)
    R = np.stack([p.restrict(e, d) for e in np.eye(nf)], 1)
    P = np.stack([p.prolongate_add(e, np.zeros(nf), d + 1) for e in np.eye(nc)], 1)
    X = X + P @ _approx_inverse(p, d + 1, rho, ncoarse) @ R @ (I - A @ X)
    return X + rho * Minv @ (I - A @ X)


@pytest.mark.parametrize("shape,L,nc", [((4, 4, 4), 2, 2), ((8, 8, 3), 3, 3)])
def test_vcycle_with_walls_equals_dense_composition(shape, L, nc):
    nx, ny, nz = shape
    p = oracle.OracleProblem(nx, ny, nz, L, kv=100.0, sigma=1.0, kh=W.kh_uniform(3, nx, ny),
                             ncoarse=nc, bc_h=1, bc_v=1)
    n = nx * ny * nz
    I = np.eye(n)
    B = np.stack([p.vcycle(e, np.zeros(n)) for e in I], 1)
    B_ref = _approx_inverse(p, 0, p.rho, nc)
    assert np.abs(B - B_ref).max() < 1e-12 * np.abs(B_ref).max()


def test_solvers_with_walls_match_direct_solve():
    """The paper's boundary conditions at its CFL number 8.4 (K = (4.2 h)^2 times
    a factor in [0.5, 2] per column): both solvers reach the direct solution and
    multigrid needs fewer iterations than CG."""
    nx = ny = 32
    nz = 16
    K = (4.2 / nx) ** 2
    p = oracle.OracleProblem(nx, ny, nz, 4, kv=K * 1e4, sigma=1.0,
                             kh=K * W.kh_uniform(2, nx, ny), bc_h=1, bc_v=1)
    f = W.rhs(2, 0, nx, ny, nz)
    ref = spla.spsolve(p.scipy().tocsc(), f)
    u, it, hist, st = p.mg_solve(f, rtol=1e-10, maxit=60)
    assert st == 0 and it < 40 and (np.diff(hist) < 0).all()
    assert np.abs(u - ref).max() < 1e-8 * np.abs(ref).max()
    u2, it2, _, rt, st2 = p.pcg_solve(f, rtol=1e-10, maxit=500)
    assert st2 == 0 and rt < 1e-10 and it2 > it
    assert np.abs(u2 - ref).max() < 1e-8 * np.abs(ref).max()


def test_line_preconditioned_condition_number_with_walls():
    """Sec. 2.1.1 estimates kappa(M^-1 A) ~ 1 + 8 w^2/h^2 (~142 at nu_CFL = 8.4),
    which the periodic box attains exactly.  Walls lift the smallest eigenvalue
    (the lowest sine mode is not constant), so with walls kappa stays below that
    value and approaches it as the grid is refined.  All eigenvalues of M^-1 A lie
    in (0, 2): A and 2M - A (A with the signs of its horizontal couplings
    flipped, still diagonally dominant) are both positive definite."""
    kappas = []
    for n in (8, 16):
        nz = 3
        h = 1.0 / n
        K = (4.2 * h) ** 2
        p = oracle.OracleProblem(n, n, nz, 1, kv=0.8 * K, sigma=1.0, zfaces=W.uniform_faces(nz),
                                 kh=np.full(n * n, K), bc_h=1, bc_v=1)
        A = p.scipy().toarray()
        ev = sla.eigh(A, _block_diag_part(A, nz), eigvals_only=True)
        assert 0.0 < ev.min() and ev.max() < 2.0
        kappas.append(ev.max() / ev.min())
    assert kappas[0] < kappas[1] < 1 + 8 * 4.2**2


def test_multigrid_robust_to_cfl_number_cg_not():
    """Sec. 5.2 on the flat box (Dirichlet walls, Neumann ends): with enough
    levels the multigrid iteration count hardly changes from nu_CFL = 8.4 to
    840, while CG's grows several-fold (kappa ~ nu^2 until the walls bound it);
    with only 3 levels the coarse problem is too ill-conditioned for two
    smoothing steps at large nu, and more coarse steps restore the count."""
    mg, cg, mg3 = {}, {}, {}
    for nu in (8.4, 84.0, 840.0):
        fb = W.FlatBox(64, 16, nu, 5)
        p = oracle.OracleProblem(64, 64, 16, 5, **fb.params())
        mg[nu] = p.mg_solve(fb.rhs(), rtol=fb.rtol, maxit=200)[1]
        fb1 = W.FlatBox(64, 16, nu, 1)
        q = oracle.OracleProblem(64, 64, 16, 1, **fb1.params())
        cg[nu] = q.pcg_solve(fb1.rhs(), rtol=fb1.rtol, maxit=5000)[1]
        fb3 = W.FlatBox(64, 16, nu, 3)
        r = oracle.OracleProblem(64, 64, 16, 3, **fb3.params())
        mg3[nu] = r.mg_solve(fb3.rhs(), rtol=fb3.rtol, maxit=300)[1]
    assert max(mg.values()) <= mg[8.4] + 2 and mg[8.4] <= 12
    assert cg[84.0] > 2 * cg[8.4] and cg[8.4] > 4 * mg[8.4]
    assert mg3[840.0] > 5 * mg[840.0]
    fb = W.FlatBox(64, 16, 840.0, 3, ncoarse=30)
    p = oracle.OracleProblem(64, 64, 16, 3, **fb.params())
    assert p.mg_solve(fb.rhs(), rtol=fb.rtol, maxit=300)[1] <= mg[840.0] + 1


def test_rowwise_forms_with_walls_equal_csr():
    nx, ny, nz = 8, 6, 7
    kh = W.kh_uniform(8, nx, ny)
    p = oracle.OracleProblem(nx, ny, nz, 2, kv=300.0, sigma=1.0, kh=kh, bc_h=1)
    q = oracle.OracleProblem(nx, ny, nz, 2, kv=300.0, sigma=1.0, kh=kh, bc_h=1, matfree=True)
    x = W.uniform_pm1(8, 1, nx * ny * nz)
    rows = np.arange(nx * ny * nz, dtype=np.int64)
    assert np.array_equal(q.apply_rows(rows, x), p.spmv(x))
    cols = np.arange(nx * ny, dtype=np.int64)
    assert np.array_equal(q.line_solve_columns(cols, x), p.line_solve(x))


def test_bc_h_validation():
    with pytest.raises(ValueError):
        oracle.OracleProblem(4, 4, 4, 1, bc_h=2)
    with pytest.raises(ValueError):
        oracle.OracleProblem(4, 4, 4, 1, bc_h=-1)
