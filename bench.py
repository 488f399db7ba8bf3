#!/usr/bin/env python3
"""Benchmark of the tensor-product multigrid / line-CG path on one MI355X.

Workload: one GPU's share at real shape, 1024 x 1024 x 128 = 134,217,728
unknowns, doubly periodic, quadratically graded vertical grid, K_v = 1e4,
per-column K_T ~ U[0.5, 2] (seed 2), sigma = 1, f ~ U[-1, 1]; 6 levels.

One step = the whole hot path once on the resident input, every solve from
u = 0 to a relative residual of 1e-8:
  1. FP64 multigrid, V(1,1) cycles (Algorithm 1);
  2. FP64 CG with the vertical line preconditioner (fused kernels);
  3. mixed precision: FP32 V-cycles inside FP64 iterative refinement;
  4. mixed precision: flexible CG (FP64) preconditioned by one FP32 V-cycle.
value = sum over the four solves of (unknowns x iterations) / step time.

The dominant kernel's roofline comes from the library's own per-kernel HIP
event timing over the timed region (gmg_timing_*), on the stream the kernels
run on.  One extra untimed step with every kernel timed picks the dominant
kernel and gives the breakdown; in the timed steps only that kernel kind is
bracketed by events, so the instrumentation does not slow the others.  The CPU baseline times the FP64 oracle (CSR) on a bounded sample of
the same workload: ten V-cycles and 36 line-PCG iterations from u = 0.
Beside the step the line reports the solve from host memory (the paper's
"total solution time") and flexible CG with the FP32 line preconditioner.
`--cfl-sweep` runs the CFL robustness study of the paper's flat box instead.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solve time & HBM GB/s (frac of peak) for MG/CG; mixed-prec vs FP64 to 1e-8"
HBM_PEAK_GBS = 8000.0

# algorithmic words per cell of the level a kernel runs on (intermediates of
# the line solves and horizontal halos stay on chip; per-column coefficients
# are amortised over the column)
WORDS_PER_CELL = {
    "spmv": 2.0,             # read x, write y
    "residual": 3.0,         # read u, f, write r   (+0.5 with the FP32 copy)
    "line_solve": 2.0,       # read r, write z
    "smooth": 3.0,           # read u, f, write u'
    "restrict_smooth": 6.0,  # per COARSE cell: read 4 fine r, write f_c, u_c
    # (inside the V-cycle each coarse level starts with a scaled line solve,
    # timed as line_solve of that level)
    "prolongate": 2.25,      # per FINE cell: read/write u_f, read 1/4 u_c
    # line-PCG's direction step alternates: odd iterations read z, p, q and
    # write p', q (5 words); even ones also take the two pending steps of the
    # iterate, reading u and the direction before last and writing u (8)
    "cg_spmv": 6.5,
    "cg_tridiag": 4.0,       # read r, q, write r, z
    "correct": 4.0,          # read u, f (8 B), e (4 B), write u (8 B), r (4 B): 32 B
    "residual_restrict": 2.25,  # per FINE cell: read u, f, write 1/4 f_c
    "prolong_smooth": 3.25,  # read u, f, write u', read 1/4 u_c (u + P u_c not stored)
    # the three vector kernels of a flexible-CG iteration with an FP32
    # preconditioner move 96 B per cell together on average: <z,q> reads z
    # (4 B) and q; the direction kernel reads z, p, q, r and writes p, q
    # (44 B), on even iterations also reading u and the direction before last
    # and writing u (68 B); the update reads r, q and writes r and its FP32
    # copy (28 B).  They share one timing kind, so each launch counts as a
    # third of the iteration.
    "fcg": 96.0 / 3.0 / 8.0,
}

SOLVES = ("mg_f64", "pcg_f64", "mg_mixed", "fcg_mixed")

# HBM traffic per launch of a kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch averaged over the kernel's
# dispatches) scaled by what the same counters read for a plain copy of known
# size.  Reported only while the kernel source hashes to the recorded value.
MEASURED_TRAFFIC = {
    # k_cg_p1 (both forms), 64x8 workgroups, tile groups of 8 (the stored
    # launch shape); profiles/cg_p1_1024x1024x128_pmc.md.  Averages over the
    # 162 dispatches that did the work (82 odd-iteration, 80 even-iteration
    # forms; the two enqueued past convergence return at once).  Plain-copy
    # calibration: 2 GiB read + 2 GiB written read FETCH_SIZE 1048592.3 KiB,
    # WRITE_SIZE 2097192.6 KiB.
    ("cg_spmv", 0, "f64"): {
        "fetch_kib": 2249939.0212,
        "write_kib": 2615226.2820,
        "copy_fetch_scale": 2097152.0 / 1048592.3438,
        "copy_write_scale": 2097152.0 / 2097192.5625,
        "source_sha256": "dd7b0d13b8c51558879fab40ede78327423d077c36128b4dd5adb5d4bc1ea7cd",
        "shape": [8, 8],
    },
}
KERNEL_SOURCE = os.path.join(ROOT, "paper_1402_3545_amd", "csrc", "kernels.hip")
COPY_PROBE_BYTES = 2 << 30   # per direction


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, level, prec, w):
    nx, ny, nz = w.nx >> level, w.ny >> level, w.nz
    esize = 8 if prec == "f64" or kernel == "fcg" else 4
    cells = nx * ny * nz
    if kernel == "prolongate":          # timed under the coarse level
        cells = (nx * 2) * (ny * 2) * nz
    words = WORDS_PER_CELL.get(kernel)
    if words is None:
        return None
    return words * cells * esize


def source_sha256():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(key, shape):
    """Counter-derived bytes per launch, or None when the kernel source or its
    launch shape differ from those the counters were taken with."""
    rec = MEASURED_TRAFFIC.get(key)
    if rec is None or rec["source_sha256"] != source_sha256() or list(shape) != rec["shape"]:
        return None
    return (rec["fetch_kib"] * 1024.0 * rec["copy_fetch_scale"] +
            rec["write_kib"] * 1024.0 * rec["copy_write_scale"])


def copy_probe(torch, reps=5):
    """A plain streaming copy of COPY_PROBE_BYTES (2 GiB read + 2 GiB written,
    far above the caches) by torch's elementwise kernel: the counter
    calibration for the traffic figures.  Returns GB/s of read + write bytes."""
    n = COPY_PROBE_BYTES // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * COPY_PROBE_BYTES / (ms / 1e3) / 1e9


def copy_ceiling(torch, G, reps=5):
    """The achievable-copy ceiling: the library's streaming copy kernel
    (gmg_copy_probe) over COPY_PROBE_BYTES, timed with HIP events on the
    current stream.  Returns GB/s of read + write bytes."""
    n = COPY_PROBE_BYTES // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    G.gmg_copy_probe(src, dst)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        G.gmg_copy_probe(src, dst)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    ok = bool(torch.equal(src[:: 1 << 20], dst[:: 1 << 20]))
    del src, dst
    torch.cuda.empty_cache()
    if not ok:
        raise RuntimeError("copy probe produced wrong values")
    return 2 * COPY_PROBE_BYTES / (ms / 1e3) / 1e9


ORACLE_REF_RTOL = 1e-10   # tolerance of the oracle solves the GPU solutions are compared with


def _rel(a, b):
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else float(np.linalg.norm(a))


def cpu_baseline(w, f, kh, zf, mg_cycles=10, cg_iters=36, share=None, largest=None,
                 batch=None):
    """The CPU leg: the FP64 oracle (CSR, OpenMP rows) timed on a bounded
    sample of the same workload -- `mg_cycles` multigrid V-cycles and
    `cg_iters` line-PCG iterations from u = 0 on the full grid; value =
    unknowns x (cycles + iterations) / time, as for the GPU line -- and the
    oracle's verdict on the GPU solutions the run produced:
      share:   {solve: u} on the same grid: the error against one oracle FP64
               multigrid solve to ORACLE_REF_RTOL, and the true FP64 residual;
      largest: (workload, f, kh, {solve: u}) on 2048^2 x 128: the true FP64
               residual by the matrix-free oracle (its CSR does not fit);
      batch:   [(workload, rhs index, f, u)]: per sampled pair, the error
               against an oracle FP64 multigrid solve and the true residual.
    Returns (baseline object, checks)."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    p = oracle.OracleProblem(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma, zfaces=zf,
                             kh=kh)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it_mg, hist_mg, _ = p.mg_solve(f, rtol=1e-300, maxit=mg_cycles)
    t_mg = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it_cg, _, _, _ = p.pcg_solve(f, rtol=1e-300, maxit=cg_iters)
    t_cg = time.perf_counter() - t0
    base = {
        "value": w.unknowns * (it_mg + it_cg) / (t_mg + t_cg),
        "unit": "unknowns*iterations/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"{it_mg} FP64 V(1,1) cycles ({t_mg:.1f} s, relres {hist_mg[-1]:.2e}) and "
                   f"{it_cg} FP64 line-PCG iterations ({t_cg:.1f} s) of the CSR oracle from u = 0 "
                   f"on the full {w.nx}x{w.ny}x{w.nz} workload; CSR assembly {t_asm:.1f} s "
                   f"excluded"),
    }
    checks = {}
    nf = float(np.linalg.norm(f))
    if share:
        log(f"[bench] oracle reference solve of {w.name} to {ORACLE_REF_RTOL:g}")
        t0 = time.perf_counter()
        u_ref, it_ref, hist_ref, st_ref = p.mg_solve(f, rtol=ORACLE_REF_RTOL, maxit=80)
        t_ref = time.perf_counter() - t0
        out = {"reference": {"solver": "oracle FP64 multigrid (CSR)", "rtol": ORACLE_REF_RTOL,
                             "iters": it_ref, "relres": float(hist_ref[-1]), "status": st_ref,
                             "s": round(t_ref, 1)}}
        for name, u in share.items():
            r = p.residual(f, u)
            out[name] = {"err_vs_oracle": _rel(u, u_ref),
                         "max_err_vs_oracle": float(np.abs(u - u_ref).max() /
                                                    np.abs(u_ref).max()),
                         "oracle_relres": float(np.linalg.norm(r)) / nf}
            log(f"[bench] {name}: error vs oracle {out[name]['err_vs_oracle']:.2e}, oracle "
                f"relres {out[name]['oracle_relres']:.2e}")
        checks[w.name] = out
        del u_ref
    del p
    if largest:
        lw, lf, lkh, sols = largest
        log(f"[bench] oracle true residuals on {lw.name} (matrix-free rows)")
        q = oracle.OracleProblem(lw.nx, lw.ny, lw.nz, lw.nlevels, kv=lw.kv, sigma=lw.sigma,
                                 zfaces=lw.zfaces(), kh=lkh, matfree=True)
        lnf = float(np.linalg.norm(lf))
        out = {}
        for name, u in sols.items():
            out[name] = {"oracle_relres": q.residual_norm2_rows(lf, u) ** 0.5 / lnf}
            log(f"[bench] {name}: oracle relres {out[name]['oracle_relres']:.2e}")
        if "mg_f64" in sols and "mg_mixed" in sols:
            out["mg_mixed"]["err_vs_fp64_mg"] = _rel(sols["mg_mixed"], sols["mg_f64"])
        checks[lw.name] = out
        del q
    if batch:
        log(f"[bench] oracle reference solves of {len(batch)} batched pairs")
        out = {}
        for bw, r, bf, u in batch:
            q = oracle.OracleProblem(bw.nx, bw.ny, bw.nz, bw.nlevels, kv=bw.kv, sigma=bw.sigma,
                                     zfaces=bw.zfaces(), kh=bw.kh())
            u_ref, it_ref, hist_ref, _ = q.mg_solve(bf, rtol=ORACLE_REF_RTOL, maxit=80)
            out[f"{bw.name}/rhs{r}"] = {
                "err_vs_oracle": _rel(u, u_ref),
                "oracle_relres": float(np.linalg.norm(q.residual(bf, u)) / np.linalg.norm(bf)),
                "oracle_iters": it_ref}
            del q, u_ref
        checks["batched"] = {"pairs": out,
                             "max_err_vs_oracle": max(v["err_vs_oracle"] for v in out.values()),
                             "max_oracle_relres": max(v["oracle_relres"] for v in out.values())}
        log(f"[bench] batched sample: max error vs oracle "
            f"{checks['batched']['max_err_vs_oracle']:.2e}")
    return base, checks


def cfl_sweep(args, torch):
    """Robustness of the solvers to the horizontal CFL number (Sec. 5.2): the
    flat box with Dirichlet side walls and Neumann ends on n^2 x nz, for each
    nu_CFL of the sweep the line-preconditioned CG and FP64 multigrid with 5,
    7 and 10 levels (coarsest 32^2, 8^2, 1^2 at n = 512), with the paper's
    coarse smoothing counts and, where those differ from two, also with two.
    Every solve starts from u = 0, runs to a relative residual of 1e-5 on the
    resident input, and is timed with HIP events after one untimed solve.
    Prints one JSON object per solve."""
    import numpy as np

    import paper_1402_3545_amd as G
    import workloads as W
    n, nz = args.cfl_n, args.cfl_nz
    depth_levels = [L for L in (5, 7, 10) if n % (1 << (L - 1)) == 0]
    table = None
    rows = []

    def timed_solve(ctx, fd, ud, fn):
        ud.zero_()
        fn()
        ud.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        it, rel, _, st = fn()
        b.record()
        b.synchronize()
        return it, rel, st, a.elapsed_time(b)

    for nu in W.CFL_SWEEP:
        configs = [("pcg_f64", 1, 2)]
        for L in depth_levels:
            nc = W.paper_coarse_sweeps(L, nu)
            configs.append(("mg_f64", L, nc))
            if nc != 2:
                configs.append(("mg_f64", L, 2))
        for solver, L, nc in configs:
            fb = W.FlatBox(n, nz, nu, L, ncoarse=nc)
            ctx = G.GmgContext(n, n, nz, L, **fb.params())
            if table is None:
                deep = G.GmgContext(n, n, nz, max(depth_levels), **fb.params())
                table, stored = G.tuned(deep, reps=3)
                log(f"[cfl] launch shapes: {'stored' if stored else 'autotuned'}")
                if args.tune_out:
                    with open(args.tune_out, "w") as fh:
                        json.dump({G.launch_key(deep): table}, fh, indent=1, sort_keys=True)
                del deep
            G.apply_launch_table(ctx, table)
            fd, ud = ctx.to_device(fb.rhs()), ctx.empty()
            if solver == "pcg_f64":
                fn = lambda: G.pcg_solve(ctx, fd, ud, fb.rtol, 50000, check=False)
            else:
                fn = lambda: G.gmg_solve(ctx, fd, ud, fb.rtol, 300, check=False)
            it, rel, st, ms = timed_solve(ctx, fd, ud, fn)
            rec = {"workload": fb.name, "nu_cfl": nu, "solver": solver, "levels": L,
                   "coarse_sweeps": nc, "iters": it, "relres": rel, "status": st,
                   "ms": round(ms, 3), "ms_per_iter": round(ms / max(it, 1), 4)}
            if nu == 8.4 and L in (1, 5):
                # the paper's "total solution time" definition at its main CFL
                # number: from host memory, copies and layout conversion included
                uh = np.zeros(fb.unknowns)
                method = "pcg" if solver == "pcg_f64" else "mg"
                G.gmg_solve_host(ctx, fb.rhs(), uh, method, fb.rtol, 50000)
                uh[:] = 0.0
                it_h, _, tm_h, st_h = G.gmg_solve_host(ctx, fb.rhs(), uh, method, fb.rtol, 50000)
                rec["host_solution"] = {"iters": it_h, "status": st_h,
                                        "total_ms": round(sum(tm_h.values()), 3),
                                        **{k + "_ms": round(v, 3) for k, v in tm_h.items()}}
            rows.append(rec)
            print(json.dumps(rec), flush=True)
            log(f"[cfl] nu {nu:g} {solver} L{L} nc{nc}: {it} it, {ms:.1f} ms, status {st}")
            del ctx, fd, ud
            torch.cuda.synchronize()
    return rows


# Sec. 5.1, Table SingleGPUTiming (one M2090, nu_CFL = 8.4, tolerance 1e-5):
# iterations, time per iteration and total solution time in ms by n_x.
PAPER_SINGLE_GPU = {
    "pcg": {128: (70, 2.8, 217.1), 256: (62, 7.5, 543.7), 512: (59, 29.7, 2029.0),
            768: (58, 65.0, 4365.0)},
    "mg": {128: (9, 12.8, 135.5), 256: (8, 27.3, 285.7), 512: (8, 88.8, 949.9)},
}


def paper_table(args, torch):
    """The paper's single-GPU table on its own model problem: the flat box with
    Dirichlet side walls at nu_CFL = 8.4, n_z = 128, 5 levels, tolerance 1e-5,
    for each n_x of the table: line-PCG and FP64 multigrid on resident data
    (one untimed and one timed solve), and the total solution time from host
    memory (copies and layout conversion included).  One JSON object per
    (solver, n_x), the paper's figures beside ours."""
    import numpy as np

    import paper_1402_3545_amd as G
    import workloads as W
    for n in (128, 256, 512, 768):
        fb = W.FlatBox(n, 128, 8.4, 5)
        ctx = G.GmgContext(n, n, fb.nz, fb.nlevels, **fb.params())
        G.tuned(ctx, reps=3)
        f = fb.rhs()
        fd, ud = ctx.to_device(f), ctx.empty()
        for solver in ("pcg", "mg"):
            if n not in PAPER_SINGLE_GPU[solver]:
                continue
            fn = ((lambda: G.pcg_solve(ctx, fd, ud, fb.rtol, 5000)) if solver == "pcg"
                  else (lambda: G.gmg_solve(ctx, fd, ud, fb.rtol, 100)))
            times = []
            for _ in range(2):
                ud.zero_()
                a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                it, rel, _, st = fn()
                e.record()
                e.synchronize()
                times.append(a.elapsed_time(e))
            uh = np.zeros_like(f)
            G.gmg_solve_host(ctx, f, uh, solver, fb.rtol, 5000)
            uh[:] = 0.0
            it_h, _, tm_h, _ = G.gmg_solve_host(ctx, f, uh, solver, fb.rtol, 5000)
            p_it, p_titer, p_total = PAPER_SINGLE_GPU[solver][n]
            rec = {"workload": fb.name, "solver": solver, "n_x": n, "iters": it,
                   "relres": rel, "status": st, "solve_ms": round(times[-1], 3),
                   "t_iter_ms": round(times[-1] / max(it, 1), 4),
                   "total_solution_ms": round(sum(tm_h.values()), 3),
                   "copy_and_layout_ms": round(sum(v for k, v in tm_h.items()
                                                   if k != "solve"), 3),
                   "paper_m2090": {"iters": p_it, "t_iter_ms": p_titer,
                                   "total_solution_ms": p_total}}
            print(json.dumps(rec), flush=True)
            log(f"[table] n {n} {solver}: {it} it (paper {p_it}), t_iter "
                f"{rec['t_iter_ms']:.3f} ms (paper {p_titer}), total "
                f"{rec['total_solution_ms']:.1f} ms (paper {p_total})")
        del ctx, fd, ud
        torch.cuda.synchronize()


def _timed(torch, fn):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    res = fn()
    b.record()
    b.synchronize()
    return res, a.elapsed_time(b)


def largest_comparison(torch, reps=2):
    """The largest single-GPU grid (2048^2 x 128, K_v = 1e5, lognormal K, 7
    levels): FP64 multigrid against FP32 V-cycles inside FP64 refinement, each
    from u = 0 to 1e-8 on the resident input, one untimed and `reps` timed
    solves (median).  Returns (record, f, kh, {solve: solution on the host})."""
    import numpy as np

    import paper_1402_3545_amd as G
    import workloads as W
    w = W.LARGEST
    log(f"[bench] generating inputs for {w.name}")
    kh, zf, f = w.kh(), w.zfaces(), w.rhs()
    rec = {"workload": w.name, "unknowns": w.unknowns, "levels": w.nlevels, "rtol": w.rtol}
    sols = {}
    for tag, prec in (("mg_f64", G.GMG_F64), ("mg_mixed", G.GMG_F32)):
        ctx = G.GmgContext(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma, zfaces=zf, kh=kh,
                           prec_precond=prec)
        _, stored = G.tuned(ctx, reps=3)
        fd, ud = ctx.to_device(f), ctx.empty()
        times = []
        for q in range(1 + reps):
            ud.zero_()
            (it, rel, _, st), ms = _timed(torch, lambda: G.gmg_solve(ctx, fd, ud, w.rtol, 100,
                                                                      check=False))
            if q:
                times.append(ms)
        ms = float(np.median(times))
        rec[tag] = {"iters": it, "ms": round(ms, 3), "relres": rel, "status": st,
                    "unknowns_iterations_per_s": w.unknowns * it / (ms / 1e3),
                    "launch_shapes": "stored" if stored else "autotuned"}
        log(f"[bench] {w.name} {tag}: {it} it, {ms:.1f} ms, relres {rel:.2e}")
        sols[tag] = ctx.from_device(ud)
        del fd, ud
        ctx.close()
        torch.cuda.empty_cache()
    rec["mixed_vs_fp64_mg_speedup"] = rec["mg_f64"]["ms"] / rec["mg_mixed"]["ms"]
    return rec, f, kh, sols


def batched_comparison(torch, sample_every=8):
    """The batched workload (64 instances of seeded sizes, 4 right-hand sides
    each, FP32 V-cycles in FP64 refinement to 1e-8): one untimed and one timed
    batched solve on resident inputs, against the same pairs solved one at a
    time by single-instance contexts -- plain FP64 multigrid, and FP32-cycle
    refinement -- with default launch shapes, one untimed solve per instance
    first, every solve timed with HIP events and the times summed.  Returns
    (record, sampled pairs for the oracle: [(workload, rhs, f, u)])."""
    import numpy as np

    import paper_1402_3545_amd as G
    import workloads as W
    insts = W.batched_instances()
    nrhs = insts[0].nrhs
    kws = [dict(nx=w.nx, ny=w.ny, nz=w.nz, nlevels=w.nlevels, kv=w.kv, sigma=w.sigma,
                zfaces=w.zfaces(), kh=w.kh()) for w in insts]
    b = G.GmgBatch(kws, nrhs=nrhs)
    fs, us = [], []
    for q, w in enumerate(insts):
        for r in range(nrhs):
            fs.append(b.to_device(w.rhs(r), q))
            us.append(b.empty(q))
    log(f"[batched] {len(insts)} instances x {nrhs} rhs, "
        f"{sum(w.unknowns for w in insts) * nrhs:.3e} unknown-rhs pairs on the device")
    times = []
    for _ in range(2):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        (it, rel, st), ms = _timed(torch, lambda: G.gmg_batch_solve(b, fs, us, rtol=1e-8,
                                                                     maxit=60))
        times.append(ms)
    sizes = np.repeat([w.unknowns for w in insts], nrhs)
    work = float((sizes * it).sum())
    rec = {"workload": f"batched-{len(insts)}x{nrhs}", "unknown_rhs": int(sizes.sum()),
           "status": st, "ms": round(times[-1], 3), "iters_min": int(it.min()),
           "iters_max": int(it.max()), "iters_mean": round(float(it.mean()), 2),
           "max_relres": float(rel.max()),
           "unknowns_iterations_per_s": work / (times[-1] / 1e3)}
    log(f"[batched] {times[-1]:.1f} ms, cycles {it.min()}-{it.max()}, "
        f"{rec['unknowns_iterations_per_s']:.3e} unknowns*it/s")
    picks = [(q, (q // sample_every) % nrhs) for q in range(0, len(insts), sample_every)]
    sample = [(insts[q], r, None, b.from_device(us[q * nrhs + r], q)) for q, r in picks]
    # the same pairs one at a time; the FP64 solutions also give every
    # batched pair's distance to the plain FP64 solve
    errs = []
    for tag, prec in (("fp64_single", G.GMG_F64), ("mixed_single", G.GMG_F32)):
        total, its, rels, bad = 0.0, [], [], 0
        for q, w in enumerate(insts):
            ctx = G.GmgContext(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma,
                               zfaces=kws[q]["zfaces"], kh=kws[q]["kh"], prec_precond=prec)
            if ctx.layout(0) != b.layout(q):
                raise RuntimeError("single-instance and batched layouts differ")
            ud = torch.zeros(b.layout(q)[1], dtype=torch.float64, device="cuda")
            G.gmg_solve(ctx, fs[q * nrhs], ud, 1e-8, 60, check=False)
            for r in range(nrhs):
                ud.zero_()
                (i1, r1, _, s1), ms = _timed(torch, lambda: G.gmg_solve(
                    ctx, fs[q * nrhs + r], ud, 1e-8, 60, check=False))
                total += ms
                its.append(i1)
                rels.append(r1)
                bad += s1 != 0
                if prec == G.GMG_F64:
                    ub = us[q * nrhs + r]
                    errs.append(float(torch.linalg.vector_norm(ub - ud) /
                                      torch.linalg.vector_norm(ud)))
            del ud
            ctx.close()
        work1 = float((sizes * np.array(its)).sum())
        rec[tag] = {"ms": round(total, 3), "iters_mean": round(float(np.mean(its)), 2),
                    "max_relres": float(np.max(rels)), "failed": int(bad),
                    "unknowns_iterations_per_s": work1 / (total / 1e3)}
        rec[f"batched_vs_{tag}_speedup"] = total / times[-1]
        log(f"[batched] {tag}: {total:.1f} ms summed over {len(its)} solves "
            f"(batched is {total / times[-1]:.2f}x faster)")
        torch.cuda.empty_cache()
    rec["max_err_vs_fp64_single"] = max(errs)
    b.close()
    del fs, us
    torch.cuda.empty_cache()
    sample = [(w, r, w.rhs(r), u) for w, r, _, u in sample]
    return rec, sample


def batched_run(args, torch):
    """`--batched`: the batched comparison alone (one JSON object)."""
    rec, _ = batched_comparison(torch)
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (for profiler runs)")
    ap.add_argument("--solves", default=",".join(SOLVES),
                    help="comma list of solves per step (profiler runs); the reported "
                         "value is only the whole-path figure with all four")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the plain copy used to calibrate traffic counters")
    ap.add_argument("--tune", choices=("auto", "off", "force"), default="auto",
                    help="launch shapes: stored table or autotune (auto), defaults (off), "
                         "always autotune (force); done before the warm-up, untimed")
    ap.add_argument("--tune-out", default=None,
                    help="write the launch-shape table of this run (JSON) to this path")
    ap.add_argument("--paper-table", action="store_true",
                    help="only run the paper's single-GPU table on its flat box (one JSON "
                         "object per solver and size)")
    ap.add_argument("--batched", action="store_true",
                    help="only run the batched workload (one JSON object)")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the largest-grid and batched comparisons after the step "
                         "(for profiler runs)")
    ap.add_argument("--workload", choices=("share", "small", "largest"), default="share",
                    help="share: 1024^2 x 128 (the default line); small: 64^3 (cache "
                         "resident); largest: 2048^2 x 128 (no CPU baseline: its CSR "
                         "does not fit the host)")
    ap.add_argument("--cfl-sweep", action="store_true",
                    help="only run the CFL robustness sweep on the flat box with Dirichlet "
                         "side walls (one JSON object per solve)")
    ap.add_argument("--cfl-n", type=int, default=512, help="horizontal size of the sweep")
    ap.add_argument("--cfl-nz", type=int, default=128, help="layers of the sweep")
    args = ap.parse_args()
    solves = [x for x in args.solves.split(",") if x]
    if any(x not in SOLVES for x in solves) or not solves:
        ap.error(f"--solves takes a comma list from {SOLVES}")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              "single-GPU by design", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.cfl_sweep:
        cfl_sweep(args, torch)
        return
    if args.batched:
        batched_run(args, torch)
        return
    if args.paper_table:
        paper_table(args, torch)
        return
    if args.copy_probe:
        gbs = copy_probe(torch)
        print(json.dumps({"copy_probe_bytes_read": COPY_PROBE_BYTES,
                          "copy_probe_bytes_written": COPY_PROBE_BYTES, "gbs": gbs}), flush=True)
        return

    import paper_1402_3545_amd as G
    import workloads as W

    w = {"share": W.SHARE, "small": W.SMALL, "largest": W.LARGEST}[args.workload]
    log(f"[bench] generating inputs for {w.name}")
    kh, zf, f = w.kh(), w.zfaces(), w.rhs()
    ctx64 = G.GmgContext(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma, zfaces=zf, kh=kh,
                         prec_precond=G.GMG_F64)
    ctx32 = G.GmgContext(w.nx, w.ny, w.nz, w.nlevels, kv=w.kv, sigma=w.sigma, zfaces=zf, kh=kh,
                         prec_precond=G.GMG_F32)
    fd = ctx64.to_device(f)
    ud = ctx64.empty()
    torch.cuda.synchronize()

    # launch shapes (untimed setup)
    shapes, store = {}, {}
    for tag, c in (("f64", ctx64), ("mixed", ctx32)):
        if args.tune == "off":
            src = "defaults"
        elif args.tune == "force":
            G.gmg_autotune(c, reps=3)
            src = "autotuned"
        else:
            _, stored = G.tuned(c, reps=3)
            src = "stored" if stored else "autotuned"
        table = G.launch_table(c)
        store[G.launch_key(c)] = table
        shapes[tag] = {"source": src, **{k: v for k, v in table.items()
                                         if k.split("/")[1] == "0"}}
        log(f"[bench] launch shapes {tag}: {src}")
    if args.tune_out:
        with open(args.tune_out, "w") as fh:
            json.dump(store, fh, indent=1, sort_keys=True)

    def step(which=None):
        out = {}
        runs = {"mg_f64": lambda: G.gmg_solve(ctx64, fd, ud, w.rtol, 100),
                "pcg_f64": lambda: G.pcg_solve(ctx64, fd, ud, w.rtol, 2000),
                "mg_mixed": lambda: G.gmg_solve(ctx32, fd, ud, w.rtol, 100),
                "fcg_mixed": lambda: G.pcg_solve(ctx32, fd, ud, w.rtol, 100, precond=1)}
        for name in (which or solves):
            fn = runs[name]
            ud.zero_()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            it, rel, _, st = fn()
            b.record()
            b.synchronize()
            out[name] = {"iters": it, "relres": rel, "status": st, "ms": a.elapsed_time(b)}
        return out

    for k in range(args.warmup):
        r = step()
        log(f"[bench] warmup {k}: " + ", ".join(f"{n} {v['iters']} it {v['ms']:.1f} ms"
                                                 for n, v in r.items()))
    def timing_table():
        table = {}
        for c in (ctx64, ctx32):
            for key, (n, ms) in G.gmg_timing_table(c).items():
                cn, cms = table.get(key, (0, 0.0))
                table[key] = (cn + n, cms + ms)
        return table

    # one untimed step with every kernel timed, solve by solve: the per-kernel
    # breakdown, each solve's algorithmic bytes, and the dominant kernel whose
    # roofline the line reports
    per_solve = {}
    for name in solves:
        for c in (ctx64, ctx32):
            G.gmg_timing_filter(c, None)
            G.gmg_timing_enable(c, True)
        step([name])
        per_solve[name] = timing_table()
        for c in (ctx64, ctx32):
            G.gmg_timing_enable(c, False)
    full = {}
    for tab in per_solve.values():
        for key, (n, ms) in tab.items():
            cn, cms = full.get(key, (0, 0.0))
            full[key] = (cn + n, cms + ms)
    dom = max((k for k in full if algorithmic_bytes(*k, w) is not None),
              key=lambda k: full[k][1])
    breakdown = {f"{k[0]}@L{k[1]}/{k[2]}": {"launches": n, "ms": round(ms, 3)}
                 for k, (n, ms) in sorted(full.items(), key=lambda kv: -kv[1][1])}

    # the timed region: HIP events bracket only the dominant kernel kind, so
    # the measurement adds no event overhead to the other kernels
    for c in (ctx64, ctx32):
        G.gmg_timing_filter(c, [dom[0]])
        G.gmg_timing_enable(c, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    table = timing_table()
    for c in (ctx64, ctx32):
        G.gmg_timing_enable(c, False)
        G.gmg_timing_filter(c, None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    last = runs[-1]
    for name, v in last.items():
        if v["status"] != 0:
            raise SystemExit(f"{name} did not converge: {v}")
    work = sum(w.unknowns * v["iters"] for v in last.values())
    value = work / (ms_per_step / 1e3)
    log(f"[bench] {args.steps} steps, {ms_per_step:.1f} ms/step: " +
        ", ".join(f"{n} {v['iters']} it {v['ms']:.1f} ms" for n, v in last.items()))

    # dominant kernel's roofline over the timed region.  The solvers enqueue
    # predicted batches of iterations and the launches past convergence return
    # at once (a few us each); where the number of launches that did the work
    # is known from the iteration counts, the average is taken over those
    # (the returned launches' few us stay in the total).
    n_dom, ms_dom = table[dom]
    n_work = n_dom
    bytes_dom = algorithmic_bytes(*dom, w)
    if dom[:2] == ("cg_spmv", 0) and all("pcg_f64" in r for r in runs):
        its = [r["pcg_f64"]["iters"] for r in runs]
        n_work = sum(its)
        # the exact mix of odd (5-word) and even (8-word) direction steps
        n_even = sum(i // 2 for i in its)
        words = (5.0 * (n_work - n_even) + 8.0 * n_even) / n_work
        bytes_dom = words * w.nx * w.ny * w.nz * 8
    avg_ms = ms_dom / n_work
    achieved = bytes_dom / (avg_ms / 1e3) / 1e9
    log("[bench] kernel breakdown (one fully timed step): " + json.dumps(breakdown))

    copy_gbs = copy_ceiling(torch, G)
    torch_copy_gbs = copy_probe(torch)
    log(f"[bench] plain-copy ceiling {copy_gbs:.0f} GB/s (library copy kernel; torch's "
        f"elementwise copy {torch_copy_gbs:.0f} GB/s)")

    # the paper's "total solution time" (Sec. 5.1): the FP64 multigrid solve
    # from host memory, copies and layout conversion included; reported beside
    # the line, never as value
    host = None
    if "mg_f64" in solves:
        # a caller's guess array holds written pages (np.zeros_like would hand
        # over untouched ones, whose first writes fault inside the copy out);
        # the second call is reported (the first also allocates the context's
        # device fields and pinned staging and is the first DMA through them)
        uh = np.full_like(f, 0.0)
        G.gmg_solve_host(ctx64, f, uh, "mg", w.rtol, 100)
        uh[:] = 0.0
        it_h, rel_h, tm_h, st_h = G.gmg_solve_host(ctx64, f, uh, "mg", w.rtol, 100)
        total = sum(tm_h.values())
        host = {"solve": "mg_f64", "iters": it_h, "relres": rel_h, "total_ms": round(total, 3),
                **{k + "_ms": round(v, 3) for k, v in tm_h.items()},
                "unknowns_iterations_per_s": w.unknowns * it_h / (total / 1e3)}
        log(f"[bench] solve from host memory: {total:.1f} ms total "
            f"({', '.join(f'{k} {v:.1f}' for k, v in tm_h.items())})")
        del uh
    # flexible CG with the FP32 line preconditioner alone: reported beside the
    # step (one untimed and one timed solve), against the FP64 line-PCG
    line_fcg = None
    if "pcg_f64" in solves:
        times = []
        for _ in range(2):
            ud.zero_()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            it_l, rel_l, _, st_l = G.pcg_solve(ctx32, fd, ud, w.rtol, 2000, precond=2)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        line_fcg = {"iters": it_l, "ms": round(times[-1], 3), "relres": rel_l, "status": st_l,
                    "fp64_pcg_ms_over_this": last["pcg_f64"]["ms"] / times[-1]}
        log(f"[bench] FP32-line flexible CG: {it_l} it, {times[-1]:.1f} ms")
    prec_id = 0 if dom[2] == "f64" else 1
    traffic = (measured_traffic(dom, G.gmg_get_launch(ctx64, dom[0], dom[1], prec_id))
               if w is W.SHARE else None)

    # each solve's algorithmic traffic: the kernels' algorithmic bytes
    # (WORDS_PER_CELL) summed over its launches in the fully timed step, over
    # its median time in the timed steps (reductions, fills and the final
    # update of the CG iterate are left out: a few words per solve)
    solve_rates = {}
    for name, v in last.items():
        ms_med = float(np.median([r[name]["ms"] for r in runs]))
        nbytes = sum(n * algorithmic_bytes(*k, w) for k, (n, _) in per_solve[name].items()
                     if algorithmic_bytes(*k, w) is not None)
        gbs = nbytes / (ms_med / 1e3) / 1e9
        solve_rates[name] = {
            "unknowns_iterations_per_s": w.unknowns * v["iters"] / (ms_med / 1e3),
            "algorithmic_gb": nbytes / 1e9,
            "algorithmic_gbs": gbs,
            "frac_of_peak": gbs / HBM_PEAK_GBS,
            "words_per_cell_iteration": nbytes / (8.0 * w.unknowns * max(v["iters"], 1)),
        }

    # the final solutions of the four solves (one more untimed solve each),
    # for the oracle's verdict in the CPU leg
    share_sols = None
    want_oracle = not args.no_cpu_baseline and w is not W.LARGEST
    if want_oracle:
        share_sols = {}
        runs_final = {"mg_f64": lambda: G.gmg_solve(ctx64, fd, ud, w.rtol, 100),
                      "pcg_f64": lambda: G.pcg_solve(ctx64, fd, ud, w.rtol, 2000),
                      "mg_mixed": lambda: G.gmg_solve(ctx32, fd, ud, w.rtol, 100),
                      "fcg_mixed": lambda: G.pcg_solve(ctx32, fd, ud, w.rtol, 100, precond=1)}
        for name in solves:
            ud.zero_()
            runs_final[name]()
            share_sols[name] = ctx64.from_device(ud)

    # the other configurations of the metric, on the same GPU: the largest
    # grid (FP64 multigrid against FP32-cycle refinement) and the batched
    # workload against the same pairs solved one at a time in plain FP64
    largest = batched = largest_host = batch_sample = None
    if w is W.SHARE and not args.no_comparisons:
        del fd, ud
        ctx64.close()
        ctx32.close()
        torch.cuda.empty_cache()
        largest, lf, lkh, lsols = largest_comparison(torch)
        largest_host = (W.LARGEST, lf, lkh, lsols) if want_oracle else None
        batched, batch_sample = batched_comparison(torch)
        if not want_oracle:
            batch_sample = None
        # bandwidth estimates: the per-cell, per-iteration algorithmic bytes
        # of the same solves on the share (its per-kernel tables), applied to
        # the other grids' unknowns x iterations (their hierarchies have the
        # same structure; coarse levels add under 2 %)
        def est(rate, name):
            if name not in solve_rates:
                return None
            gbs = rate * solve_rates[name]["words_per_cell_iteration"] * 8.0 / 1e9
            return {"algorithmic_gbs_estimate": gbs, "frac_of_peak_estimate": gbs / HBM_PEAK_GBS,
                    "bytes_per_cell_iteration_from": f"{name} on the share"}
        try:
            for tag in ("mg_f64", "mg_mixed"):
                e = est(largest[tag]["unknowns_iterations_per_s"], tag)
                if e:
                    largest[tag].update(e)
            e = est(batched["unknowns_iterations_per_s"], "mg_mixed")
            if e:
                batched.update(e)
        except (KeyError, TypeError) as ex:  # an estimate never costs the line
            log(f"[bench] bandwidth estimates skipped: {ex!r}")

    base = checks = None
    if want_oracle:
        log("[bench] timing the CPU oracle sample")
        base, checks = cpu_baseline(w, f, kh, zf, share=share_sols, largest=largest_host,
                                    batch=batch_sample)
        log(f"[bench] oracle: {base['value']:.3e} unknowns*it/s on {base['cores']} threads")

    def speedup(a, b):
        if a not in last or b not in last or last[b]["ms"] <= 0:
            return None
        return last[a]["ms"] / last[b]["ms"]

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "nx": w.nx, "ny": w.ny, "nz": w.nz, "levels": w.nlevels, "kv": w.kv,
            "kh": {"uniform": "U[0.5,2]", "lognormal": "exp(0.5 N(0,1))",
                   "const": "1"}[w.kh_model] + f" seed {w.seed}", "rtol": w.rtol,
            "step": ("FP64 MG + FP64 line-CG + FP32-cycle MG in FP64 refinement + FP64 "
                     "flexible CG with FP32 V-cycle, each from u=0"),
            "solves_run": solves,
        },
        "solves": {n: {"iters": v["iters"], "ms": round(v["ms"], 3),
                       "ms_median": round(float(np.median([r[n]["ms"] for r in runs])), 3),
                       "relres": v["relres"], **solve_rates[n]} for n, v in last.items()},
        "solves_note": ("algorithmic_gbs: the solve's kernels' algorithmic bytes (words per "
                        "cell of each kernel x launches) over its median time; relres is the "
                        "library's FP64 true relative residual"),
        "mixed_vs_fp64_mg_speedup": speedup("mg_f64", "mg_mixed"),
        "fcg_mixed_vs_fp64_mg_speedup": speedup("mg_f64", "fcg_mixed"),
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom[0]} level {dom[1]} {dom[2]}",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_source": ("stored: rocprofv3 FETCH_SIZE/WRITE_SIZE of this kernel source "
                               "and launch shape, copy-calibrated (profiles/)"
                               if traffic is not None else None),
            "copy_ceiling_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "torch_copy_gbs": torch_copy_gbs,
            "avg_ms": avg_ms,
            "launches": n_dom,
            "launches_doing_work": n_work,
            "algorithmic_bytes": bytes_dom,
        },
        "kernel_breakdown_ms": breakdown,
        "kernel_breakdown_note": ("one untimed step with every kernel bracketed by HIP events; "
                                  "in the timed steps only the dominant kernel is"),
        "launch_shapes": shapes,
        "host_solution": host,
        "fcg_line_mixed": line_fcg,
        "cpu_baseline": base,
        "oracle_checks": checks,
        "largest": largest,
        "batched": batched,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
