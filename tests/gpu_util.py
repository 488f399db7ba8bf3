"""Shared helpers of the GPU parity tests: problem construction for both the
HIP library and the CPU oracle from the same seeded inputs, and comparison
bars.  Imports torch lazily so CPU-only collection works."""

from __future__ import annotations

import numpy as np

import oracle
import workloads as W


def problem(nx, ny, nz, nlevels=1, kv=1e3, seed=3, kh_model="uniform", bc_v=0, ncoarse=2,
            prec_precond=0, matfree=False, bc_h=0, kscale=1.0, zfaces=None):
    """(library context, oracle problem, kh) for one operator."""
    import paper_1402_3545_amd as G
    if kh_model == "uniform":
        kh = W.kh_uniform(seed, nx, ny)
    elif kh_model == "lognormal":
        kh = W.kh_lognormal(seed, nx, ny)
    else:
        kh = W.kh_constant(nx, ny)
    kh = kh * kscale
    zf = W.quadratic_faces(nz) if zfaces is None else zfaces
    ctx = G.GmgContext(nx, ny, nz, nlevels, kv=kv, sigma=1.0, zfaces=zf, kh=kh, bc_v=bc_v,
                       ncoarse=ncoarse, prec_precond=prec_precond, bc_h=bc_h)
    orc = oracle.OracleProblem(nx, ny, nz, nlevels, kv=kv, sigma=1.0, zfaces=zf, kh=kh,
                               bc_v=bc_v, ncoarse=ncoarse, matfree=matfree, bc_h=bc_h)
    return ctx, orc, kh


def abs_matvec(orc, x, depth=0):
    """|A| |x| (row-wise bound of the terms summed in A x)."""
    A = orc.scipy(depth)
    A.data = np.abs(A.data)
    return A @ np.abs(x)


def device_index(ctx, rows, level=0):
    """Library-layout indices of canonical rows (j*nx+i)*nz+k."""
    nx, ny, nz = ctx.shape(level)
    ldx, _ = ctx.layout(level)
    rows = np.asarray(rows, dtype=np.int64)
    k = rows % nz
    col = rows // nz
    i = col % nx
    j = col // nx
    return (j * nz + k) * ldx + i


def max_rel(got, ref, scale):
    return float(np.max(np.abs(got - ref) / scale))


def f32_line_bar(nz):
    """Bar of the FP32 line kernels against the FP64 oracle on FP32-rounded
    inputs, relative to max|z|: about seven FP32 unit roundoffs per layer
    (4e-7 nz), at least 2e-6.  tests/test_f32_line_bar.py shows that a textbook
    FP32 Thomas sweep on these operators' columns stays well inside it."""
    return max(2e-6, 4e-7 * nz)
