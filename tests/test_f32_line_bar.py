"""Where the FP32 line-kernel bar comes from (CPU).

The GPU parity tests hold the FP32 line kernels (line solve, Smooth,
ResSmooth) to f32_line_bar(nz) of max|z| against the FP64 oracle on
FP32-rounded inputs.  This test runs the textbook Thomas algorithm (forward
elimination, back substitution; the Thomas solve of Sec. 2.2 per column) in
FP32 arithmetic on the FP32-rounded columns of the operators the tests and
workloads use, and checks that the bar leaves a stated margin above that
sweep's own error: an FP32 kernel is held to what a plain FP32 elimination
achieves, not to something looser."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import f32_line_bar

# the bar must exceed a textbook FP32 Thomas sweep's error by this factor
MARGIN = 1.5


def _columns(nx, ny, nz, kv, kh_model, seed):
    """Tridiagonal diagonal blocks of A (sub, diag, super per column) from the
    oracle's CSR rows, canonical order (column-major blocks of nz rows)."""
    kh = W.kh_uniform(seed, nx, ny) if kh_model == "uniform" else W.kh_lognormal(seed, nx, ny)
    p = oracle.OracleProblem(nx, ny, nz, 1, kv=kv, sigma=1.0, zfaces=W.quadratic_faces(nz),
                             kh=kh)
    A = p.scipy(0).tocsr()
    n = nx * ny * nz
    rows = np.arange(n)
    d = np.asarray(A[rows, rows]).reshape(-1)
    lo = np.zeros(n)
    up = np.zeros(n)
    k = rows % nz
    has_lo, has_up = k > 0, k < nz - 1
    lo[has_lo] = np.asarray(A[rows[has_lo], rows[has_lo] - 1]).reshape(-1)
    up[has_up] = np.asarray(A[rows[has_up], rows[has_up] + 1]).reshape(-1)
    ncol = nx * ny
    return p, lo.reshape(ncol, nz), d.reshape(ncol, nz), up.reshape(ncol, nz)


def _thomas(lo, d, up, r, dtype):
    """Textbook Thomas algorithm in `dtype` arithmetic, all columns at once."""
    lo, d, up, r = (a.astype(dtype) for a in (lo, d, up, r))
    nz = d.shape[1]
    c = np.zeros_like(d)
    g = np.zeros_like(d)
    c[:, 0] = up[:, 0] / d[:, 0]
    g[:, 0] = r[:, 0] / d[:, 0]
    for k in range(1, nz):
        m = d[:, k] - lo[:, k] * c[:, k - 1]
        c[:, k] = up[:, k] / m
        g[:, k] = (r[:, k] - lo[:, k] * g[:, k - 1]) / m
    z = np.zeros_like(d)
    z[:, nz - 1] = g[:, nz - 1]
    for k in range(nz - 2, -1, -1):
        z[:, k] = g[:, k] - c[:, k] * z[:, k + 1]
    return z


@pytest.mark.parametrize("nz,kv,kh_model", [
    (128, 1e3, "uniform"),    # the GPU tests' operator at the maximum height
    (128, 1e4, "uniform"),    # the one-GPU-share workload
    (128, 1e5, "lognormal"),  # the largest workload
    (64, 1e3, "uniform"),     # the small workload's height
    (37, 1e3, "uniform"),     # a ragged height of the GPU tests
])
def test_f32_line_bar_exceeds_textbook_fp32_thomas(nz, kv, kh_model):
    nx = ny = 8
    p, lo, d, up = _columns(nx, ny, nz, kv, kh_model, seed=3)
    r = W.uniform_pm1(3, 2, nx * ny * nz).astype(np.float32).astype(np.float64)
    z64 = p.line_solve(r).reshape(nx * ny, nz)   # FP64 oracle, canonical order
    # the FP64 oracle agrees with an FP64 Thomas on the same blocks
    assert np.max(np.abs(_thomas(lo, d, up, r.reshape(-1, nz), np.float64) - z64)) \
        <= 1e-13 * np.max(np.abs(z64))
    z32 = _thomas(lo, d, up, r.reshape(-1, nz), np.float32).astype(np.float64)
    err = np.max(np.abs(z32 - z64)) / np.max(np.abs(z64))
    assert err > 0.0
    assert f32_line_bar(nz) >= MARGIN * err, (nz, kv, err, f32_line_bar(nz))
    # and the bar is not slack beyond what FP32 rounding over nz layers explains
    assert f32_line_bar(nz) <= 50.0 * max(err, 2e-7 * nz / 8), (nz, err)
