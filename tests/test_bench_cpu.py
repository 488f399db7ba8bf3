"""The benchmark's host-side contract, on the CPU: one GPU only, argument
checks, the CPU-baseline leg and the tables the roofline figures use."""

import importlib.util
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", BENCH)
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no benchmark line


def test_unknown_solve_is_rejected():
    r = subprocess.run([sys.executable, BENCH, "--solves", "mg_f64,nope"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "--solves" in r.stderr


def test_cpu_baseline_times_the_oracle_on_a_sample():
    b = _bench_module()
    nx, ny, nz, L = 16, 16, 8, 2
    w = SimpleNamespace(nx=nx, ny=ny, nz=nz, nlevels=L, kv=1e3, sigma=1.0,
                        unknowns=nx * ny * nz)
    kh = W.kh_uniform(3, nx, ny)
    zf = W.quadratic_faces(nz)
    f = W.uniform_pm1(3, 1, nx * ny * nz)
    out, checks = b.cpu_baseline(w, f, kh, zf, mg_cycles=2, cg_iters=3)
    assert out["kind"] == "oracle" and out["unit"] == "unknowns*iterations/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "2 FP64 V(1,1) cycles" in out["sample"] and "3 FP64 line-PCG" in out["sample"]
    assert checks == {}


def test_cpu_leg_judges_solutions_by_the_oracle():
    """The oracle checks of the CPU leg: a solution to 1e-8 is close to the
    reference solve and has a true residual below 1e-8; a perturbed one is
    reported as such (on a tiny instance, with the oracle's own solutions
    standing in for the GPU's)."""
    import oracle
    b = _bench_module()
    w = W.Workload("tiny-16x16x8", 16, 16, 8, 2, 1e3, 1.0, 3, "uniform", 1e-8)
    kh, zf, f = w.kh(), w.zfaces(), w.rhs()
    p = oracle.OracleProblem(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma, zfaces=zf,
                             kh=kh)
    u8, _, _, _ = p.mg_solve(f, rtol=1e-8, maxit=60)
    bad = u8 * (1.0 + 1e-3)
    w2 = W.Workload("tiny-matfree", 16, 16, 8, 2, 1e3, 1.0, 3, "uniform", 1e-8)
    _, checks = b.cpu_baseline(w, f, kh, zf, mg_cycles=1, cg_iters=1,
                               share={"good": u8, "bad": bad},
                               largest=(w2, f, kh, {"mg_f64": u8, "mg_mixed": bad}),
                               batch=[(w, 0, f, u8)])
    share = checks[w.name]
    assert share["reference"]["relres"] < b.ORACLE_REF_RTOL
    assert share["good"]["oracle_relres"] < 1e-8 and share["good"]["err_vs_oracle"] < 1e-6
    assert share["bad"]["err_vs_oracle"] == __import__("pytest").approx(1e-3, rel=1e-3)
    big = checks[w2.name]
    assert big["mg_f64"]["oracle_relres"] < 1e-8
    assert big["mg_mixed"]["err_vs_fp64_mg"] == __import__("pytest").approx(1e-3, rel=1e-6)
    pair = checks["batched"]["pairs"][f"{w.name}/rhs0"]
    assert pair["err_vs_oracle"] < 1e-6 and pair["oracle_relres"] < 1e-8


def test_roofline_tables():
    import paper_1402_3545_amd as G
    b = _bench_module()
    # every kernel kind of the per-kernel breakdown that moves field data has
    # its algorithmic words per cell
    for k in G.KERNELS:
        if k in ("reduce", "aux", "fcg"):
            continue
        assert k in b.WORDS_PER_CELL, k
    assert b.WORDS_PER_CELL["cg_spmv"] == 6.5   # 5 and 8 words on alternate iterations
    assert b.WORDS_PER_CELL["prolong_smooth"] == 3.25
    for key, rec in b.MEASURED_TRAFFIC.items():
        assert len(rec["shape"]) == 2 and rec["fetch_kib"] > 0 and rec["write_kib"] > 0
        # FETCH_SIZE counts a 128-byte read request as 64 bytes on gfx950, so a
        # plain copy reads about half its bytes (some boxes a little less)
        assert 1.9 < rec["copy_fetch_scale"] < 2.7 and 0.9 < rec["copy_write_scale"] < 1.1
        assert len(rec["source_sha256"]) == 64
    # the counters are used only while the kernel source is the one measured
    rec = b.MEASURED_TRAFFIC[("cg_spmv", 0, "f64")]
    got = b.measured_traffic(("cg_spmv", 0, "f64"), rec["shape"])
    if b.source_sha256() == rec["source_sha256"]:
        assert got == np.float64(rec["fetch_kib"] * 1024 * rec["copy_fetch_scale"] +
                                 rec["write_kib"] * 1024 * rec["copy_write_scale"])
    else:
        assert got is None
    assert b.measured_traffic(("cg_spmv", 0, "f64"), [rec["shape"][0], 99]) is None
