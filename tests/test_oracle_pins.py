"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms
(the flat-box stencil and the condition number of Sec. 2.1.1, the Fourier
symbol of the periodic operator), library routines (dense LU, Cholesky, sparse
direct solves, generalised eigenvalues), exactness properties (linear
functions under the vertical flux and the bilinear prolongation), finite
termination of CG, and the dense composition of Algorithm 1.
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _canon(nx, ny, nz):
    """Index map (i, j, k) -> canonical row (j*nx + i)*nz + k."""
    return lambda i, j, k: (j * nx + i) * nz + k


def _dense(p, d=0):
    return p.scipy(d).toarray()


def _block_diag_part(A, nz):
    n = A.shape[0]
    blk = np.arange(n) // nz
    return np.where(blk[:, None] == blk[None, :], A, 0.0)


# ---------------------------------------------------------------------------
# Generator
# ---------------------------------------------------------------------------

def test_splitmix64_published_outputs(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    for seed, stream, idx, hexv in rows:
        got = W.splitmix64(int(seed), int(stream), int(idx), 1)[0]
        assert int(got) == int(hexv, 16)


def test_generator_is_counter_based():
    a = W.splitmix64(7, 3, 0, 1000)
    b = W.splitmix64(7, 3, 400, 10)
    assert np.array_equal(a[400:410], b)
    u = W.uniform01(3, 1, 100000)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


# ---------------------------------------------------------------------------
# Assembly
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc_v", [0, 1])
def test_flat_box_stencil_closed_form(bc_v):
    """Sec. 2.1.1: on an equidistant grid with constant coefficients each row,
    divided by the cell volume, is  1 + 4 w^2/h^2 + 2 w^2 l^2/h_z^2  on the
    diagonal, -w^2/h^2 to each horizontal and -w^2 l^2/h_z^2 to each vertical
    neighbour (here K = w^2, K_v = w^2 l^2, sigma = 1).  End rows lose one
    vertical neighbour; a Dirichlet end face half a layer away adds 2 K_v/h_z^2."""
    nx, ny, nz = 6, 6, 5
    K, Kv, sig = 0.37, 2.9, 1.0
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=Kv, sigma=sig, zfaces=W.uniform_faces(nz),
                             kh=np.full(nx * ny, K), bc_v=bc_v)
    A = _dense(p)
    h, hz = 1.0 / nx, 1.0 / nz
    vol = h * h * hz
    idx = _canon(nx, ny, nz)
    for j in range(ny):
        for i in range(nx):
            for k in range(nz):
                g = idx(i, j, k)
                row = A[g] / vol
                vert = 2 * Kv / hz**2
                if k in (0, nz - 1):
                    vert = (3 if bc_v == 0 else 1) * Kv / hz**2
                assert row[g] == pytest.approx(sig + 4 * K / h**2 + vert, rel=1e-12)
                for (a, b) in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    gn = idx((i + a) % nx, (j + b) % ny, k)
                    assert row[gn] == pytest.approx(-K / h**2, rel=1e-12)
                if k > 0:
                    assert row[g - 1] == pytest.approx(-Kv / hz**2, rel=1e-12)
                if k < nz - 1:
                    assert row[g + 1] == pytest.approx(-Kv / hz**2, rel=1e-12)
                assert np.count_nonzero(row) == 5 + (k > 0) + (k < nz - 1)


def test_flat_box_stencil_on_coarse_levels():
    """Coarse levels rediscretise the same operator with h doubled and the
    column coefficient averaged over the four children (Sec. 3.1: the column
    coefficients depend on the multigrid level).  With K alternating K1, K2 from
    column to column in x, every coarse column has K = (K1 + K2)/2 and the
    coarse rows again follow the flat-box closed form of Sec. 2.1.1."""
    nx, ny, nz, L = 16, 16, 4, 3
    K1, K2, Kv = 0.3, 1.9, 2.0
    kh = np.where(np.arange(nx)[None, :] % 2 == 0, K1, K2) * np.ones((ny, 1))
    p = oracle.OracleProblem(nx, ny, nz, L, kv=Kv, sigma=1.0, zfaces=W.uniform_faces(nz),
                             kh=kh.reshape(-1), bc_v=1)
    hz = 1.0 / nz
    for d in (1, 2):
        A = _dense(p, d)
        cx, cy = nx >> d, ny >> d
        hx, hy = 1.0 / cx, 1.0 / cy
        vol = hx * hy * hz
        Kbar = 0.5 * (K1 + K2)
        idx = _canon(cx, cy, nz)
        for (i, j, k) in ((0, 0, 1), (cx - 1, cy - 1, 2), (1, 2 % cy, 0)):
            g = idx(i, j, k)
            row = A[g] / vol
            vert = (2 if 0 < k < nz - 1 else 1) * Kv / hz**2
            assert row[g] == pytest.approx(1.0 + 2 * Kbar / hx**2 + 2 * Kbar / hy**2 + vert,
                                           rel=1e-12)
            assert row[idx((i + 1) % cx, j, k)] == pytest.approx(-Kbar / hx**2, rel=1e-12)
            assert row[idx(i, (j + 1) % cy, k)] == pytest.approx(-Kbar / hy**2, rel=1e-12)


def test_single_column_periodic_level_is_the_vertical_operator():
    """A periodic level of one column is its own neighbour in every direction:
    the horizontal fluxes vanish and each row is |T| (sigma dz_k + vertical
    terms), i.e. the flat-box stencil of Sec. 2.1.1 without its horizontal part
    (here |T| = 1)."""
    nz, Kv = 5, 2.0
    p = oracle.OracleProblem(4, 4, nz, 3, kv=Kv, sigma=1.3, zfaces=W.uniform_faces(nz),
                             kh=W.kh_uniform(2, 4, 4), bc_v=0)
    assert p.shape(2) == (1, 1, nz)
    A = _dense(p, 2)
    hz = 1.0 / nz
    for k in range(nz):
        vert = (3 if k in (0, nz - 1) else 2) * Kv / hz**2
        assert A[k, k] / hz == pytest.approx(1.3 + vert, rel=1e-12)
        for m in range(nz):
            if abs(m - k) == 1:
                assert A[k, m] / hz == pytest.approx(-Kv / hz**2, rel=1e-12)
            elif m != k:
                assert A[k, m] == 0.0


@pytest.mark.parametrize("shape", [(4, 4, 8), (2, 6, 3), (8, 4, 5), (6, 2, 2)])
def test_symmetric_m_matrix_and_cholesky(shape):
    nx, ny, nz = shape
    kh = 0.5 + 1.5 * W.uniform01(11, 0, nx * ny)
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=1e3, sigma=1.0, kh=kh)
    A = _dense(p)
    assert np.array_equal(A, A.T)                      # bitwise symmetric
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all() and (np.diag(A) > 0).all()  # M-matrix sign pattern
    assert (A.sum(axis=1) > 0).all()                   # strict diagonal dominance (sigma > 0)
    np.linalg.cholesky(A)                              # positive definite


def test_vertical_flux_exact_for_linear_profiles():
    """Finite-volume fluxes are exact for linear functions: with Neumann ends
    and u = zeta (cell-centre height, constant in the horizontal), interior
    rows of A u reduce to the zero-order term |T| sigma dz_k zeta_k on any
    graded grid; u = 1 gives |T| sigma dz_k in every row."""
    nx, ny, nz = 4, 4, 9
    zf = W.quadratic_faces(nz)
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=37.0, sigma=0.8, zfaces=zf,
                             kh=0.5 + W.uniform01(3, 0, nx * ny), bc_v=1)
    dz = np.diff(zf)
    zc = 0.5 * (zf[:-1] + zf[1:])
    area = 1.0 / (nx * ny)
    scale = area * 37.0 / dz.min()      # size of the terms that cancel
    y1 = p.spmv(np.ones(nx * ny * nz)).reshape(nx * ny, nz)
    assert np.allclose(y1, area * 0.8 * dz[None, :], rtol=0, atol=1e-13 * scale)
    yz = p.spmv(np.tile(zc, nx * ny)).reshape(nx * ny, nz)
    expect = area * 0.8 * dz * zc
    assert np.allclose(yz[:, 1:-1], expect[None, 1:-1], rtol=0, atol=1e-12 * scale)


def test_fourier_symbol_of_periodic_operator():
    """For constant K and an input phi_theta(i,j) v_k with phi = cos(tx i + ty j),
    A(phi v) = phi [B0 v + K lam(theta) dz * v], with B0 the operator on
    horizontally constant inputs and lam = (hy/hx)(2-2cos tx) + (hx/hy)(2-2cos ty)."""
    nx, ny, nz = 8, 6, 7
    K = 1.7
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=50.0, sigma=1.3, kh=np.full(nx * ny, K))
    dz = np.diff(W.quadratic_faces(nz))
    hx, hy = 1.0 / nx, 1.0 / ny
    rng = np.random.default_rng(0)
    v = rng.standard_normal(nz)
    B0v = p.spmv(np.tile(v, nx * ny)).reshape(ny, nx, nz)[0, 0]
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
    for mx, my in ((1, 0), (0, 2), (3, 1), (4, 3)):
        tx, ty = 2 * math.pi * mx / nx, 2 * math.pi * my / ny
        phi = np.cos(tx * ii + ty * jj)                        # (ny, nx)
        x = (phi[:, :, None] * v[None, None, :]).reshape(-1)
        lam = (hy / hx) * (2 - 2 * math.cos(tx)) + (hx / hy) * (2 - 2 * math.cos(ty))
        expect = phi[:, :, None] * (B0v + K * lam * dz * v)[None, None, :]
        got = p.spmv(x).reshape(ny, nx, nz)
        assert np.allclose(got, expect, rtol=0, atol=1e-12 * np.abs(B0v).max())


def test_manufactured_solution_second_order():
    """u* = sin(2 pi x) cos(2 pi y) sin(pi z) solves -K Lap u - K_v u_zz + sigma u = g
    with g = (8 pi^2 K + pi^2 K_v + sigma) u* (periodic in x, y; zero at z = 0, 1).
    With b = cell volume * g(centre) the max-norm error falls at second order on
    the quadratically graded grid."""
    K, Kv, sig = 1.0, 1.0, 1.0
    errs = []
    for n in (8, 16, 32):
        nz = n
        zf = W.quadratic_faces(nz)
        p = oracle.OracleProblem(n, n, nz, 1, kv=Kv, sigma=sig, zfaces=zf)
        xc = (np.arange(n) + 0.5) / n
        zc = 0.5 * (zf[:-1] + zf[1:])
        dz = np.diff(zf)
        X = xc[None, :, None]
        Y = xc[:, None, None]
        Z = zc[None, None, :]
        ustar = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * np.sin(np.pi * Z)
        g = (8 * np.pi**2 * K + np.pi**2 * Kv + sig) * ustar
        b = (g * dz[None, None, :] / (n * n)).reshape(-1)
        u = spla.spsolve(p.scipy().tocsc(), b)
        errs.append(np.abs(u - ustar.reshape(-1)).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 1.85 and min(orders) > 1.6, (errs, orders)


def test_manufactured_solution_across_coefficient_jumps():
    """K = K1 on x < 1/2, K2 on x > 1/2 (periodic, so jumps at x = 0 and 1/2).
    u* = sin(2 pi x)/K(x) sin(pi z) is continuous with continuous flux K u_x, and
    solves -div(K grad u) - K_v u_zz + sigma u = g with
    g = (4 pi^2 sin(2 pi x) + (pi^2 K_v + sigma) sin(2 pi x)/K) sin(pi z).
    Only a face coefficient that keeps the flux exact across the jump (the
    harmonic mean) keeps the error second order."""
    K1, K2, Kv, sig = 1.0, 10.0, 1.0, 1.0
    errs = []
    for n in (8, 16, 32):
        nz = 8
        zf = W.uniform_faces(nz)
        xc = (np.arange(n) + 0.5) / n
        Kx = np.where(xc < 0.5, K1, K2)
        kh = np.tile(Kx, n)
        p = oracle.OracleProblem(n, n, nz, 1, kv=Kv, sigma=sig, zfaces=zf, kh=kh)
        zc = 0.5 * (zf[:-1] + zf[1:])
        sx = np.sin(2 * np.pi * xc)
        ustar = (sx / Kx)[None, :, None] * np.sin(np.pi * zc)[None, None, :] * np.ones((n, 1, 1))
        gx = 4 * np.pi**2 * sx + (np.pi**2 * Kv + sig) * sx / Kx
        g = gx[None, :, None] * np.sin(np.pi * zc)[None, None, :] * np.ones((n, 1, 1))
        b = (g * np.diff(zf)[None, None, :] / (n * n)).reshape(-1)
        u = spla.spsolve(p.scipy().tocsc(), b)
        # vertical error is fixed by nz; remove it by comparing with the solve of the
        # same discrete vertical operator: refine only horizontally and difference
        errs.append(u.reshape(n, n, nz))
    # horizontal convergence: compare successive grids at coarse cell centres
    d1 = np.abs(errs[0] - 0.25 * sum(errs[1][b::2, a::2] for a in (0, 1) for b in (0, 1))).max()
    d2 = np.abs(errs[1] - 0.25 * sum(errs[2][b::2, a::2] for a in (0, 1) for b in (0, 1))).max()
    assert math.log2(d1 / d2) > 1.7, (d1, d2)


# ---------------------------------------------------------------------------
# Line solve and condition number
# ---------------------------------------------------------------------------

def test_line_solve_matches_dense_lu():
    nx, ny, nz = 4, 4, 8
    kh = W.kh_uniform(5, nx, ny)
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=1e4, sigma=1.0, kh=kh)
    A = _dense(p)
    M = _block_diag_part(A, nz)
    r = W.uniform_pm1(5, 1, nx * ny * nz)
    z = p.line_solve(r)
    ref = np.linalg.solve(M, r)
    assert np.abs(z - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("grid", ["uniform", "quadratic"])
def test_condition_number_matches_paper(golden_dir, grid):
    """Sec. 2.1.1, eq. (ConditionNumber): kappa(M^-1 A) = 1 + 8 w^2/h^2 for the
    flat box with vertical Neumann ends; with w = 4.2 h the paper quotes ~142.
    On the periodic box the formula is exact for even n and any vertical grid."""
    row = [l.split() for l in open(os.path.join(golden_dir, "condition_number.txt"))
           if l.strip() and not l.startswith("#")][0]
    nu, w_over_h, kappa_paper = float(row[0]), float(row[1]), float(row[2])
    assert w_over_h == pytest.approx(nu / 2)
    n, nz = 8, 4
    h = 1.0 / n
    w2 = (w_over_h * h) ** 2
    zf = W.uniform_faces(nz) if grid == "uniform" else W.quadratic_faces(nz)
    p = oracle.OracleProblem(n, n, nz, 1, kv=w2 * 0.9, sigma=1.0, zfaces=zf,
                             kh=np.full(n * n, w2), bc_v=1)
    A = _dense(p)
    M = _block_diag_part(A, nz)
    ev = sla.eigh(A, M, eigvals_only=True)
    kappa = ev.max() / ev.min()
    assert kappa == pytest.approx(1 + 8 * w_over_h**2, rel=1e-9)
    assert round(kappa) == kappa_paper


def test_condition_number_drops_fourfold_per_level():
    """Sec. 3 (coarse grid solver): the condition number of each coarser level
    is smaller by the square of the grid-spacing ratio.  On the periodic flat
    box with Neumann ends kappa_l - 1 = 8 K/(h_l^2 sigma) exactly, so doubling
    h divides kappa - 1 by 4 on every level of the hierarchy."""
    n, nz, L = 16, 3, 3
    K = (4.2 / n) ** 2
    p = oracle.OracleProblem(n, n, nz, L, kv=0.5 * K, sigma=1.0, zfaces=W.uniform_faces(nz),
                             kh=np.full(n * n, K), bc_v=1)
    kap = []
    for d in range(L):
        A = _dense(p, d)
        ev = sla.eigh(A, _block_diag_part(A, nz), eigvals_only=True)
        kap.append(ev.max() / ev.min())
    assert kap[0] == pytest.approx(1 + 8 * 4.2**2, rel=1e-9)
    for d in range(1, L):
        assert (kap[d] - 1) == pytest.approx((kap[0] - 1) / 4**d, rel=1e-9)


def test_condition_number_dirichlet_closed_form():
    """With Dirichlet ends the same Fourier argument gives
    kappa = 1 + 8K / (h^2 (sigma + s_min)), s_min the smallest eigenvalue of the
    vertical operator S relative to diag(dz); sigma + s_min is read off the
    operator on horizontally constant inputs."""
    n, nz, K = 6, 5, 0.02
    zf = W.quadratic_faces(nz)
    p = oracle.OracleProblem(n, n, nz, 1, kv=3.0, sigma=1.0, zfaces=zf, kh=np.full(n * n, K))
    h = 1.0 / n
    B0 = np.stack([p.spmv(np.tile(e, n * n)).reshape(n * n, nz)[0] for e in np.eye(nz)], 1)
    c_min = sla.eigh(B0, h * h * np.diag(np.diff(zf)), eigvals_only=True).min()
    A = _dense(p)
    ev = sla.eigh(A, _block_diag_part(A, nz), eigvals_only=True)
    assert ev.max() / ev.min() == pytest.approx(1 + 8 * K / (h * h * c_min), rel=1e-9)


# ---------------------------------------------------------------------------
# Inter-grid transfers
# ---------------------------------------------------------------------------

def test_restriction_on_deltas_and_sums():
    nx, ny, nz = 4, 6, 3
    p = oracle.OracleProblem(nx, ny, nz, 2)
    fine, coarse = _canon(nx, ny, nz), _canon(nx // 2, ny // 2, nz)
    for j in range(ny):
        for i in range(nx):
            for k in range(nz):
                e = np.zeros(nx * ny * nz)
                e[fine(i, j, k)] = 1.0
                fc = p.restrict(e)
                assert fc.sum() == 1.0 and fc[coarse(i // 2, j // 2, k)] == 1.0
    r = W.uniform_pm1(1, 1, nx * ny * nz)
    assert p.restrict(r).sum() == pytest.approx(r.sum(), rel=1e-13)
    assert np.allclose(p.restrict(np.full(nx * ny * nz, 2.5)), 10.0)


def test_prolongation_reproduces_bilinear_functions():
    """Cell-centred bilinear interpolation is exact for a + bx + cy + dxy at fine
    cells whose coarse stencil does not wrap; constants are exact everywhere."""
    nx, ny, nz = 16, 12, 2
    p = oracle.OracleProblem(nx, ny, nz, 2)
    ncx, ncy = nx // 2, ny // 2
    Xc = (np.arange(ncx) + 0.5) / ncx
    Yc = (np.arange(ncy) + 0.5) / ncy
    f = lambda x, y: 0.3 + 1.1 * x - 0.7 * y + 2.3 * x * y
    uc = np.repeat(f(Xc[None, :], Yc[:, None])[:, :, None], nz, axis=2).reshape(-1)
    uf = p.prolongate_add(uc, np.zeros(nx * ny * nz)).reshape(ny, nx, nz)
    xf = (np.arange(nx) + 0.5) / nx
    yf = (np.arange(ny) + 0.5) / ny
    ref = f(xf[None, :], yf[:, None])
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    assert np.allclose(uf[inner][..., 0], ref[inner], rtol=0, atol=1e-14)
    assert np.allclose(uf[inner][..., 1], ref[inner], rtol=0, atol=1e-14)
    one = p.prolongate_add(np.ones(ncx * ncy * nz), np.zeros(nx * ny * nz))
    assert np.allclose(one, 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("nx,ny", [(12, 8), (8, 8), (4, 6)])
def test_prolongation_is_translation_equivariant_on_periodic_grids(nx, ny):
    """On a doubly periodic grid every coarse cell is like every other, so the
    prolongation commutes with translations: shifting the coarse field by s
    cells moves the fine output by 2s cells.  The check covers every fine cell,
    in particular the first and last columns and rows whose coarse stencils
    wrap round (Sec. 2.2, cell-centred interpolation; periodic grid of the
    workloads).  The same weights meet the same values in the same order, so
    the equality is bitwise."""
    nz = 3
    p = oracle.OracleProblem(nx, ny, nz, 2)
    ncx, ncy = nx // 2, ny // 2
    uc = W.uniform_pm1(5, 1, ncx * ncy * nz).reshape(ncy, ncx, nz)
    zero = np.zeros(nx * ny * nz)
    base = p.prolongate_add(uc.reshape(-1), zero).reshape(ny, nx, nz)
    for sx, sy in [(1, 0), (0, 1), (1, 1), (ncx - 1, 0), (0, ncy - 1), (ncx - 1, ncy - 1)]:
        moved = np.roll(uc, (sy, sx), axis=(0, 1))
        out = p.prolongate_add(moved.reshape(-1), zero).reshape(ny, nx, nz)
        assert np.array_equal(out, np.roll(base, (2 * sy, 2 * sx), axis=(0, 1))), (sx, sy)


def test_prolongation_fourier_symbol_on_periodic_grids():
    """Closed form of the periodic prolongation on a Fourier mode.  For the coarse
    field Re exp(i(tx I + ty J + phi)) the 1D interpolation gives its child on the
    side s = -1 (even fine index) or s = +1 (odd) the factor (3 + exp(i s t)) / 4,
    and the 9/3/3/1 stencil over 16 is the product of the two 1D factors.  With
    t = 2 pi m / n_c the mode is periodic, so the formula holds at every fine cell,
    including those whose coarse neighbour lies across the wrap."""
    nx, ny, nz = 16, 12, 2
    p = oracle.OracleProblem(nx, ny, nz, 2)
    ncx, ncy = nx // 2, ny // 2
    I = np.arange(ncx)[None, :]
    J = np.arange(ncy)[:, None]
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    zero = np.zeros(nx * ny * nz)
    for mx, my in [(1, 0), (0, 1), (1, 1), (3, 2), (ncx - 1, 1), (ncx // 2, ncy // 2)]:
        tx, ty = 2 * math.pi * mx / ncx, 2 * math.pi * my / ncy
        phases = [0.3, 1.9]
        uc = np.stack([np.cos(tx * I + ty * J + ph) for ph in phases], axis=-1)
        out = p.prolongate_add(uc.reshape(-1), zero).reshape(ny, nx, nz)
        sx = np.where(i % 2 == 1, 1.0, -1.0)
        sy = np.where(j % 2 == 1, 1.0, -1.0)
        gx = (3.0 + np.exp(1j * sx * tx)) / 4.0
        gy = (3.0 + np.exp(1j * sy * ty)) / 4.0
        for k, ph in enumerate(phases):
            mode = np.exp(1j * (tx * (i // 2) + ty * (j // 2) + ph))
            ref = np.real(mode * gx * gy)
            assert np.allclose(out[..., k], ref, rtol=0, atol=1e-14), (mx, my, k)


# ---------------------------------------------------------------------------
# Smoothers, V-cycle, solvers
# ---------------------------------------------------------------------------

def _hier(nx, ny, nz, L, seed=3, ncoarse=2, kv=100.0):
    kh = W.kh_uniform(seed, nx, ny)
    return oracle.OracleProblem(nx, ny, nz, L, kv=kv, sigma=1.0, kh=kh, ncoarse=ncoarse)


def test_smooth_and_restrict_smooth_dense():
    p = _hier(4, 4, 6, 2)
    rho = 2.0 / 3.0
    A = _dense(p, 0)
    M = _block_diag_part(A, 6)
    f = W.uniform_pm1(1, 1, 96)
    u = W.uniform_pm1(1, 2, 96)
    ref = u + rho * np.linalg.solve(M, f - A @ u)
    assert np.allclose(p.smooth(f, u), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    Ac = _dense(p, 1)
    Mc = _block_diag_part(Ac, 6)
    fc, uc = p.restrict_smooth(f, 1)
    assert np.allclose(fc, p.restrict(f), rtol=0, atol=0)
    refc = rho * np.linalg.solve(Mc, fc)
    assert np.allclose(uc, refc, rtol=0, atol=1e-13 * np.abs(refc).max())


def _dense_transfer(p, d_coarse):
    nf, nc = p.size(d_coarse - 1), p.size(d_coarse)
    R = np.stack([p.restrict(e, d_coarse - 1) for e in np.eye(nf)], 1)
    P = np.stack([p.prolongate_add(e, np.zeros(nf), d_coarse) for e in np.eye(nc)], 1)
    return R, P


def _approx_inverse(p, d, rho, ncoarse):
    """Matrix of the cycle started on level d from a zero guess (Algorithm 1)."""
    A = _dense(p, d)
    Minv = np.linalg.inv(_block_diag_part(A, p.nz))
    I = np.eye(A.shape[0])
    X = rho * Minv
    if d == p.nlevels - 1:
        for _ in range(ncoarse - 1):
            X = X + rho * Minv @ (I - A @ X)
        return X
    R, P = _dense_transfer(p, d + 1)
    X = X + P @ _approx_inverse(p, d + 1, rho, ncoarse) @ R @ (I - A @ X)
    return X + rho * Minv @ (I - A @ X)


@pytest.mark.parametrize("shape,L,nc", [((4, 4, 4), 2, 2), ((8, 8, 3), 3, 2),
                                        ((8, 4, 3), 2, 3), ((4, 4, 3), 1, 2)])
def test_vcycle_equals_dense_composition(shape, L, nc):
    nx, ny, nz = shape
    p = _hier(nx, ny, nz, L, ncoarse=nc)
    rho = p.rho
    n = nx * ny * nz
    A = _dense(p, 0)
    I = np.eye(n)
    S = I - rho * np.linalg.solve(_block_diag_part(A, nz), A)
    E = np.stack([p.vcycle(np.zeros(n), e) for e in I], 1)
    B = np.stack([p.vcycle(e, np.zeros(n)) for e in I], 1)
    if L == 1:
        E_ref = np.linalg.matrix_power(S, nc)
        B_ref = _approx_inverse(p, 0, rho, nc)
    else:
        R, P = _dense_transfer(p, 1)
        E_ref = S @ (I - P @ _approx_inverse(p, 1, rho, nc) @ R @ A) @ S
        B_ref = _approx_inverse(p, 0, rho, nc)
    assert np.abs(E - E_ref).max() < 1e-12 * max(1.0, np.abs(E_ref).max())
    assert np.abs(B - B_ref).max() < 1e-12 * np.abs(B_ref).max()
    # the cycle is a consistent iteration: E = I - B A
    assert np.abs(E - (I - B @ A)).max() < 1e-11


def test_mg_monotone_and_matches_direct_solve():
    nx = ny = 32
    nz = 16
    p = oracle.OracleProblem(nx, ny, nz, 3, kv=1e3, sigma=1.0, kh=W.kh_uniform(2, nx, ny))
    f = W.rhs(2, 0, nx, ny, nz)
    u, it, hist, st = p.mg_solve(f, rtol=1e-10, maxit=60)
    assert st == 0 and it < 40
    assert (np.diff(hist) < 0).all()                    # monotone residual reduction
    assert hist[-1] < 1e-10
    ref = spla.spsolve(p.scipy().tocsc(), f)
    assert np.abs(u - ref).max() < 1e-8 * np.abs(ref).max()


def test_pcg_finite_termination_on_few_eigenvalues():
    """CG ends in at most as many steps as M^-1 A has distinct eigenvalues.  On a
    2x2 periodic grid with constant K the horizontal symbol takes the values
    0, 4, 8 and M^-1 A has at most 2 nz + 1 distinct eigenvalues."""
    nz = 3
    p = oracle.OracleProblem(2, 2, nz, 1, kv=10.0, sigma=1.0, kh=np.full(4, 0.7))
    f = W.uniform_pm1(9, 1, 4 * nz)
    u, it, hist, rt, st = p.pcg_solve(f, rtol=1e-11, maxit=50)
    assert st == 0 and it <= 2 * nz + 1
    assert rt < 1e-10


def test_pcg_energy_decreases_and_solves():
    nx = ny = 8
    nz = 8
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=1e3, sigma=1.0, kh=W.kh_uniform(4, nx, ny))
    A = p.scipy()
    f = W.rhs(4, 0, nx, ny, nz)
    energies = []
    for m in range(1, 12):
        u, it, _, _, _ = p.pcg_solve(f, rtol=1e-14, maxit=m)
        energies.append(0.5 * u @ (A @ u) - f @ u)
    dE = np.diff(energies)
    tol = 1e-14 * abs(energies[0])
    assert (dE[:3] < -tol).all()          # strict decrease while above rounding
    assert (dE < tol).all()               # never increases beyond rounding
    u, it, hist, rt, st = p.pcg_solve(f, rtol=1e-12, maxit=500)
    ref = np.linalg.solve(A.toarray(), f)
    assert st == 0 and rt < 1e-11
    assert np.abs(u - ref).max() < 1e-9 * np.abs(ref).max()


def test_small_workload_iteration_counts():
    """64x64x64 periodic box, K = 1, K_v = 1e3, 4 levels: MG needs far fewer
    iterations than CG (Sec. 5.1 reports < 10 vs ~60 on the paper's operator)."""
    w = W.SMALL
    p = oracle.OracleProblem(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma,
                             zfaces=w.zfaces(), kh=w.kh())
    f = w.rhs()
    _, it_mg, hist, st = p.mg_solve(f, rtol=w.rtol, maxit=50)
    _, it_cg, _, rt, st2 = p.pcg_solve(f, rtol=w.rtol, maxit=500)
    assert st == 0 and st2 == 0
    assert it_mg < 10 and it_mg < it_cg
    assert rt < w.rtol * 1.01


def test_rowwise_forms_equal_csr_forms():
    nx, ny, nz = 8, 6, 7
    kh = W.kh_uniform(8, nx, ny)
    p = oracle.OracleProblem(nx, ny, nz, 2, kv=300.0, sigma=1.0, kh=kh)
    q = oracle.OracleProblem(nx, ny, nz, 2, kv=300.0, sigma=1.0, kh=kh, matfree=True)
    x = W.uniform_pm1(8, 1, nx * ny * nz)
    f = W.uniform_pm1(8, 2, nx * ny * nz)
    rows = np.arange(nx * ny * nz)
    assert np.array_equal(q.apply_rows(rows, x), p.spmv(x))
    r = p.residual(f, x)
    assert q.residual_norm2_rows(f, x) == pytest.approx(r @ r, rel=1e-13)
    cols = np.array([0, 5, nx * ny - 1])
    z = q.line_solve_columns(cols, f)
    ref = p.line_solve(f)
    sel = q.column_rows(cols)
    assert np.array_equal(z[sel], ref[sel])
    assert np.isnan(np.delete(z, sel)).all()
    with pytest.raises(RuntimeError):
        q.spmv(x)


def test_invalid_inputs_raise():
    with pytest.raises(ValueError):
        oracle.OracleProblem(6, 6, 4, 3)      # 6 not divisible by 4
    with pytest.raises(ValueError):
        oracle.OracleProblem(4, 4, 4, 4)      # 4 not divisible by 8
    with pytest.raises(ValueError):
        oracle.OracleProblem(4, 4, 1, 1)      # nz < 2
    with pytest.raises(ValueError):
        oracle.OracleProblem(4, 4, 4, 1, kh=-np.ones(16))
    with pytest.raises(ValueError):
        oracle.OracleProblem(4, 4, 4, 1, zfaces=np.zeros(5))
