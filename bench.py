#!/usr/bin/env python3
"""Benchmark of the RKA / RKAB hot path on one MI355X.

Workload (the paper-scale configuration): A is 80000 x 10000 with iid N(0,1)
entries in FP64 (6.4 GB), planted x* ~ N(0,1), b = A x* + e with
e ~ N(0, 1e-2) (inconsistent).  Synthetic, seeded, generated on the device.

One step = one pass of the whole hot path over that system for every cell of
the grid  {RKA q in (16, 64, 256), alpha in (1, alpha*(q))}  and
{RKAB q in (16, 64, 256), block size in (10, 100), alpha = 1}: each cell is a
complete solve -- squared row norms, running sum, Philox row stream,
persistent iteration kernel -- over a fixed budget of row projections
(--rows-per-cell), so every cell moves the same number of row bytes.

Printed: one JSON line with the aggregate row projections/s of the step
(``value``), per-cell projections/s, HBM GB/s and error to the least-squares
solution, the roofline of the dominant kernel (algorithmic bytes over its
HIP-event time on the stream it runs on), and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "row projections/s + HBM GB/s; time to 1e-6 rel. error, plain FP64 vs chosen"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=80000)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--rows-per-cell", type=int, default=819200)
    ap.add_argument("--cells", default="all", help="all | rka | rkab | comma list like rkab:256:10")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plateau", action="store_true",
                    help="skip the time-to-plateau passes of the cells")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision / batching / differentiation measurements")
    ap.add_argument("--forms", default="precision,precision_200000x20000,batching,"
                    "differentiation,distributed_approach,coherent_rows")
    ap.add_argument("--batch-systems", type=int, default=512)
    ap.add_argument("--batch-sample", type=int, default=16,
                    help="systems solved one by one in plain FP64 for the batching comparison")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (the reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_cells(spec, astar):
    cells = []
    for q in (16, 64, 256):
        cells.append(("rka", q, 1, 1.0, "1"))
        cells.append(("rka", q, 1, astar[q], "alpha*"))
    for q in (16, 64, 256):
        for bs in (10, 100):
            cells.append(("rkab", q, bs, 1.0, "1"))
    if spec == "all":
        return cells
    if spec in ("rka", "rkab"):
        return [c for c in cells if c[0] == spec]
    out = []
    for item in spec.split(","):
        parts = item.split(":")
        meth, q, bs = parts[0], int(parts[1]), int(parts[2]) if len(parts) > 2 else 1
        alab = parts[3] if len(parts) > 3 else "1"
        out.append((meth, q, bs, astar[q] if alab == "alpha*" else 1.0, alab))
    return out


def kernel_name(stats, storage="double", vec=2, rkab=False, bs=1):
    """Template instance as named in the library: <storage, accumulation,
    elements per 16-byte vec, register bucket, all-gather / iterate in LDS>
    (the block kernels: <storage, elements per vec, rows per thread[, RKAB]>)."""
    acc = "float" if stats.get("accumulate") == 1 else "double"
    flag = "true" if stats.get("variant") == 1 else "false"
    if stats["kernel"] == 1:
        return f"rka_col_kernel<{storage}, {acc}, {vec}, {stats['bucket']}, {flag}>"
    if stats["kernel"] == 3:
        return f"rka_sstep_kernel<{storage}, {vec}, {stats['bucket']}, {'true' if rkab else 'false'}>"
    if stats["kernel"] == 4:
        # mode 0: RKA; RKAB: 1 with one block per outer iteration, 2 in sub-blocks
        mode = 0 if not rkab else (2 if stats["variant"] < bs else 1)
        return f"rka_blk_kernel<{storage}, {vec}, {stats['bucket']}, {mode}>"
    return f"rkab_kernel<{storage}, {acc}, {vec}, {stats['bucket']}, {flag}>"


def cpu_baseline(A, b, seconds):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    q = 16

    def timed(K):
        t0 = time.perf_counter()
        _, info = oracle.rka(A, b, q=q, alpha=1.0, max_iter=K, seed=3)
        return time.perf_counter() - t0, info

    timed(0)                       # pages A in before anything is timed
    t_setup, _ = timed(0)          # row norms + running sum over all of A
    # The sample grows until one run fills the budget, each next length from
    # the rate just measured but at most 8x longer: a setup time that varies
    # between calls cannot make the estimate run away (a difference of two
    # timings did once, giving a sample of millions of iterations)
    K = 64
    while True:
        dt, info = timed(K)
        log(f"[bench] CPU oracle baseline: {K} iterations in {dt:.1f} s")
        if dt >= 0.8 * seconds or K >= (1 << 22):
            break
        per_iter = max((dt - t_setup) / K, dt / K / 4, 1e-7)
        K = int(min(8 * K, max(2 * K, (seconds - t_setup) / per_iter)))
    return {"value": info["projections"] / dt, "unit": "row projections/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"oracle RKA (plain C, FP64, single thread) on the same {A.shape[0]}x"
                       f"{A.shape[1]} FP64 system, q={q}, alpha=1, {K} iterations "
                       f"({info['projections']} projections) including its row norms and "
                       f"running sum, {dt:.1f} s wall"),
            "host_cpu": _cpu_model(), "host_threads": os.cpu_count()}


def copy_ceiling(gib=4, reps=7):
    """STREAM-copy ceiling of this GPU in the same run: a device-to-device copy
    of `gib` GiB (torch), read + write bytes over its HIP-event time, median
    of `reps`."""
    import torch
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    ms = times[len(times) // 2]
    del src, dst
    torch.cuda.empty_cache()
    return {"gbps": 2 * n * 8 / (ms / 1e3) / 1e9, "bytes_moved": 2 * n * 8, "median_ms": ms,
            "reps": reps, "how": f"torch device-to-device copy of {gib} GiB, HIP events"}


def time_to_plateau(P, b, x_ls, cell, rate, seed, max_segments=400):
    """Time to the error plateau of one cell, with the paper's two passes
    (Sec. 3.1): pass 1 runs the cell in segments that resume the same row
    stream and measures ||x - x_LS|| / ||x_LS|| after each, until the error has
    not fallen by 1 % over the last 10 segments (a stationary error: RKA and
    RKAB stall at a horizon above x_LS on an inconsistent system, Sec. 2.3.1);
    the plateau error is the median of the last 10, and K_p the first
    iteration count whose error is within 10 % of it.  Pass 2 times a fresh
    solve of exactly K_p iterations without stopping tests (HIP events on the
    solve's stream, and wall time)."""
    import torch
    meth, q, bs, alpha, _ = cell
    method = 0 if meth == "rka" else 1
    # segment length: about 1/20 of the e-folds to a 1e-4 error reduction
    k_est = 9.2 / max(rate * (bs if method == 1 else 1), 1e-12)
    seg = max(1, int(k_est / 20))
    x = torch.zeros_like(x_ls)
    nls = float(x_ls.norm())
    errs, ks, k = [], [], 0
    for _ in range(max_segments):
        x, info, _ = P.solve(b, method=method, q=q, block_size=bs, alpha=alpha, max_iter=seg,
                             seed=seed, x0=x, iter_offset=k, raise_on_error=False)
        k += seg
        e = float((x - x_ls).norm()) / nls
        errs.append(e)
        ks.append(k)
        if info.status < 0 or not math.isfinite(e):
            return {"status": info.status, "iterations": k, "rel_err": e, "diverged": True}
        if len(errs) > 10 and errs[-1] > 0.99 * errs[-11]:
            break
    tail = sorted(errs[-10:])
    plateau = tail[len(tail) // 2]
    kp = next(kk for kk, e in zip(ks, errs) if e <= 1.1 * plateau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info, st = P.solve(b, method=method, q=q, block_size=bs, alpha=alpha, max_iter=kp,
                          seed=seed, timing=True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return {"plateau_rel_err": plateau, "iterations_to_plateau": kp, "segment": seg,
            "segments": len(errs), "rel_err_at_kp": float((x - x_ls).norm()) / nls,
            "ms_to_plateau": wall, "kernel_ms_to_plateau": st["iterate_ms"] + st["coef_ms"],
            "projections_to_plateau": info.projections}


def cpu_baseline_cells(workloads):
    """The oracle on the smaller configurations, whole: the 4000 x 200 FP64
    consistent solve to 1e-8 (q = 8, alpha = 1 and alpha*), and the forward +
    backward of the differentiable least-squares solve at 20000 x 1000 FP32
    (the GPU path's steps, each by the oracle: refined forward with the range
    projection, the minimum-norm column solve, the row solve for lambda, the
    rank-2 gradient)."""
    import numpy as np
    import oracle
    import paper_2401_17474_amd as rka  # Eq. (6) only (a host function)
    out = {}
    A, xs, _ = workloads.gaussian_system(4000, 200, seed=workloads.DATA_SEED + 1)
    b = A @ xs
    sv = np.linalg.svd(A, compute_uv=False)
    F = float(np.sum(sv ** 2))
    for name, alpha in (("alpha_1", 1.0), ("alpha_star", None)):
        a = alpha if alpha is not None else rka.alpha_star(sv[-1] ** 2 / F, sv[0] ** 2 / F, 8)
        t0 = time.perf_counter()
        x, info = oracle.rka(A, b, q=8, alpha=a, max_iter=200000, tol=1e-8, x_ref=xs, seed=3)
        dt = time.perf_counter() - t0
        out[f"4000x200_rka_q8_{name}"] = {"seconds": dt, "iterations": info["iterations"],
                                          "projections_per_s": info["projections"] / dt,
                                          "alpha": a, "status": info["status"]}
    # differentiation form, 20000 x 1000 FP32 storage
    m, n, q = 20000, 1000, 64
    A, xs, b = workloads.gaussian_system(m, n, seed=workloads.DATA_SEED + 6, noise_var=1e-2,
                                         dtype="f32")
    A = np.array(A)
    t = np.random.default_rng(workloads.DATA_SEED + 6).standard_normal(n)
    s_ext = _mp_extremes(m, n)
    al = rka.alpha_star(*s_ext, q)
    k = int(math.ceil(1.1 * 9.2 / _rate(s_ext, al, q)))
    t0 = time.perf_counter()
    x, _ = oracle.refine(A, b, q=q, acc32=1, alpha=al, inner_iters=k, range_iters=k, range_q=q,
                         range_alpha=al, sweeps=3, seed=3)
    t_fwd = time.perf_counter() - t0
    At = oracle.transpose(A)
    g = 2 * (x - t)
    z, _ = oracle.refine(At, g, q=q, acc32=0, alpha=al, inner_iters=k, sweeps=3, seed=4)
    lam, _ = oracle.refine(A, z, q=q, acc32=1, alpha=al, inner_iters=k, sweeps=3, seed=5)
    r = b - A.astype(np.float64) @ x
    dA = np.outer(r, lam) - np.outer(z, x)
    t_all = time.perf_counter() - t0
    out["20000x1000_f32_forward_backward"] = {
        "seconds": t_all, "forward_seconds": t_fwd, "q": q, "alpha": al, "inner_iters": k,
        "sweeps": 3, "dA_norm": float(np.linalg.norm(dA))}
    return out


# -- the three forms -------------------------------------------------------------

def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3


def _rate(s, alpha, q):
    """e-folds of the error per RKA iteration from the one-step identity
    E||e_{k+1}||^2 = sum_j phi(s_j) (v_j^T e_k)^2 (consistent part):
    phi(s) = 1 - 2 alpha s + alpha^2 s / q + alpha^2 (1 - 1/q) s^2, worst at an
    extreme of the spectrum."""
    rho = max(1 - 2 * alpha * x + alpha ** 2 * x / q + alpha ** 2 * (1 - 1 / q) * x * x
              for x in s)
    return -math.log(rho) / 2


def _mp_extremes(m, n):
    """Marchenko-Pastur edges of sigma^2 / ||A||_F^2 for an iid m x n matrix."""
    F = m * n
    return (math.sqrt(m) - math.sqrt(n)) ** 2 / F, (math.sqrt(m) + math.sqrt(n)) ** 2 / F


def bench_precision(rka, A, xs, b, x_ls, s_ext):
    """Plain FP64 RKA vs the precision form (BF16 / FP32 storage, FP32 inner
    solves, FP64 refinement) at 80000 x 10000: time to 1e-6 relative error on
    the planted consistent system and, horizon-free, on the least-squares
    problem; then inner-solve throughput per storage type at 200000 x 20000."""
    import torch
    out = {}
    m, n = A.shape
    q, qc = 256, 32
    al, alc = rka.alpha_star(*s_ext, q), rka.alpha_star(*s_ext, qc)
    k_in = int(math.ceil(1.1 * 9.2 / _rate(s_ext, al, q)))      # ~1e-4 per inner solve
    k_col = int(math.ceil(1.1 * 9.2 / _rate(s_ext, alc, qc)))
    A16 = A.to(torch.bfloat16)
    A32 = A.to(torch.float32)
    # consistent: b = A x*, each storage type's own rounded matrix
    cons = {}
    bc = A @ xs
    (x, info, st), ms = _timed(lambda: rka.solve_ex(A, bc, method=0, q=q, alpha=al,
                                                   max_iter=400000, tol=1e-6, x_ref=xs,
                                                   check_every=25, timing=True))
    cons["fp64_plain_rka"] = {"ms": ms, "iterations": info.iterations, "status": info.status,
                              "rel_err": info.rel_err, "q": q, "alpha": al}
    for name, Ast in (("bf16_refined", A16), ("fp32_refined", A32)):
        bst = Ast.to(torch.float64) @ xs
        (x, ri), ms = _timed(lambda: rka.refine_solve(Ast, bst, q=q, alpha=al, accumulate=1,
                                                      inner_iters=k_in, max_sweeps=6, tol=1e-6,
                                                      x_ref=xs))
        cons[name] = {"ms": ms, "sweeps": ri.sweeps, "status": ri.status,
                      "per_sweep_rel_err": ri.measures, "inner_iters": k_in,
                      "projections": ri.projections}
    for name in ("bf16_refined", "fp32_refined"):
        cons[name]["speedup_vs_fp64"] = cons["fp64_plain_rka"]["ms"] / cons[name]["ms"]
    out["consistent_80000x10000_to_1e-6"] = cons
    # least squares (b = A x* + N(0, 1e-2)): horizon-free refinement in both
    lsq = {}
    At = rka.transpose(A)
    (x, ri), ms = _timed(lambda: rka.refine_solve(A, b, At=At, q=q, alpha=al, accumulate=0,
                                                  inner_iters=k_in, range_iters=k_col,
                                                  range_q=qc, range_alpha=alc, max_sweeps=5,
                                                  tol=1e-6, x_ref=x_ls))
    lsq["fp64_horizon_free"] = {"ms": ms, "sweeps": ri.sweeps, "status": ri.status,
                                "per_sweep_rel_err": ri.measures}
    del At
    torch.cuda.empty_cache()
    A16d = A16.to(torch.float64)
    G = A16d.T @ A16d
    L = torch.linalg.cholesky(G)
    x_ls16 = torch.cholesky_solve((A16d.T @ b)[:, None], L)[:, 0]
    r = b - A16d @ x_ls16
    x_ls16 = x_ls16 + torch.cholesky_solve((A16d.T @ r)[:, None], L)[:, 0]
    del A16d, G, L, r
    torch.cuda.empty_cache()
    At16 = rka.transpose(A16)
    (x, ri), ms = _timed(lambda: rka.refine_solve(A16, b, At=At16, q=q, alpha=al, accumulate=1,
                                                  inner_iters=k_in, range_iters=k_col,
                                                  range_q=qc, range_alpha=alc, max_sweeps=5,
                                                  tol=1e-6, x_ref=x_ls16))
    lsq["bf16_horizon_free"] = {"ms": ms, "sweeps": ri.sweeps, "status": ri.status,
                                "per_sweep_rel_err": ri.measures,
                                "speedup_vs_fp64": lsq["fp64_horizon_free"]["ms"] / ms}
    lsq["inner_iters"], lsq["range_iters"], lsq["range_q"] = k_in, k_col, qc
    out["least_squares_80000x10000_to_1e-6"] = lsq
    del At16, A16, A32
    torch.cuda.empty_cache()
    # inner-solve throughput at 200000 x 20000 (A = the rounded Gaussian)
    M, N, q3, K3 = 200000, 20000, 64, 300
    gen = torch.Generator(device=A.device)
    gen.manual_seed(240117474 + 3)
    A64 = torch.randn((M, N), generator=gen, device=A.device, dtype=torch.float64)
    x3 = torch.randn(N, generator=gen, device=A.device, dtype=torch.float64)
    b3 = A64 @ x3 + 1e-2 * torch.randn(M, generator=gen, device=A.device, dtype=torch.float64)
    a3 = rka.alpha_star(*_mp_extremes(M, N), q3)
    thr = {}
    for name, dt, acc, esz in (("fp64", torch.float64, 0, 8), ("fp32", torch.float32, 1, 4),
                               ("bf16", torch.bfloat16, 1, 2)):
        As = A64 if dt == torch.float64 else A64.to(dt)
        x, info, st = rka.solve_ex(As, b3, method=0, q=q3, alpha=a3, max_iter=K3, seed=2,
                                   accumulate=acc, timing=True)
        it_s = (st["iterate_ms"] + st["coef_ms"]) / 1e3
        bpp = N * esz + 20
        y, gms = _timed(lambda: rka.gemv(As, x3, c=b3, gamma=-1.0))
        thr[name] = {"projections_per_s": info.projections / it_s,
                     "hbm_gbps": info.projections * bpp / it_s / 1e9,
                     "us_per_iteration": (st["iterate_ms"] + st["coef_ms"]) * 1e3 / K3,
                     "kernel": kernel_name(st, {"fp64": "double", "fp32": "float",
                                                "bf16": "rka::bf16_t"}[name],
                                           16 // esz),
                     "residual_gemv_gbps": M * N * esz / (gms / 1e3) / 1e9}
        if As is not A64:
            del As
        torch.cuda.empty_cache()
    out["inner_throughput_200000x20000_rka_q64"] = thr
    del A64, b3, x3
    torch.cuda.empty_cache()
    return out


def _lsq_normal_equations(Aw_rows, b, n, chunk=20000):
    """x_LS of min ||A x - b|| in FP64 from the normal equations, G = A^T A
    summed over row chunks (A widened to FP64 chunk by chunk), Cholesky, and
    one refinement step with the FP64 residual (cond(A) < 2 for these iid
    Gaussian shapes, so G is well conditioned).  A measurement aid."""
    import torch
    m = b.shape[0]
    G = torch.zeros((n, n), dtype=torch.float64, device=b.device)
    Atb = torch.zeros(n, dtype=torch.float64, device=b.device)
    for r0 in range(0, m, chunk):
        Ac = Aw_rows(r0, min(m, r0 + chunk))
        G += Ac.T @ Ac
        Atb += Ac.T @ b[r0:r0 + Ac.shape[0]]
        del Ac
    L = torch.linalg.cholesky(G)
    x = torch.cholesky_solve(Atb[:, None], L)[:, 0]
    Atr = torch.zeros(n, dtype=torch.float64, device=b.device)
    for r0 in range(0, m, chunk):
        Ac = Aw_rows(r0, min(m, r0 + chunk))
        Atr += Ac.T @ (b[r0:r0 + Ac.shape[0]] - Ac @ x)
        del Ac
    x = x + torch.cholesky_solve(Atr[:, None], L)[:, 0]
    del G, L
    return x


def bench_precision_large(rka):
    """The precision form at 200000 x 20000 (b = A x* + N(0, 1e-4)): A stored
    as BF16 (8 GB) and as FP32 (16 GB) -- each rounded matrix is the problem
    matrix -- solved to 1e-10 relative error against that matrix's FP64
    least-squares solution by horizon-free FP64 refinement around binary32
    inner solves, error reported per sweep; and the time to 1e-6 of BF16 /
    FP32 against the same refinement in plain FP64 (FP64 storage and
    arithmetic) on the FP64 matrix.  Inner solves: RKA with q = 64 and
    alpha* (Eq. (6)) from the Marchenko-Pastur edges; the range projection
    on the transposed copy with q = 8."""
    import torch
    dev = torch.device("cuda:0")
    M, N = 200000, 20000
    # q = 64 on A; q = 8 on the 200000-column transpose, whose slices leave
    # the one-iteration kernel room for 8 rows per workgroup in FP64
    q, qc = 64, 8
    s_ext = _mp_extremes(M, N)
    al, alc = rka.alpha_star(*s_ext, q), rka.alpha_star(*s_ext, qc)
    k_in = int(math.ceil(1.1 * 9.2 / _rate(s_ext, al, q)))      # ~1e-4 per inner solve
    k_col = int(math.ceil(1.1 * 9.2 / _rate(s_ext, alc, qc)))
    gen = torch.Generator(device=dev)
    gen.manual_seed(240117474 + 3)
    A64 = torch.randn((M, N), generator=gen, device=dev, dtype=torch.float64)
    xs = torch.randn(N, generator=gen, device=dev, dtype=torch.float64)
    e = 1e-2 * torch.randn(M, generator=gen, device=dev, dtype=torch.float64)
    out = {"shape": f"{M}x{N}", "noise": "N(0, 1e-4)", "q": q, "alpha": al, "range_q": qc,
           "range_alpha": alc, "inner_iters": k_in, "range_iters": k_col}
    runs = {}
    for name, dt in (("bf16", torch.bfloat16), ("fp32", torch.float32), ("fp64", torch.float64)):
        As = A64 if dt == torch.float64 else A64.to(dt)
        b = (A64 @ xs if dt == torch.float64 else
             torch.cat([As[r0:r0 + 20000].to(torch.float64) @ xs for r0 in range(0, M, 20000)]))
        b = b + e
        log(f"[bench] 200000x20000 {name}: least-squares reference")
        x_ls = _lsq_normal_equations(lambda r0, r1: As[r0:r1].to(torch.float64), b, N)
        At = rka.transpose(As)
        PA, PT = rka.Plan(As), rka.Plan(At)
        acc = 0 if dt == torch.float64 else 1
        entry = {}
        targets = (1e-6,) if dt == torch.float64 else (1e-6, 1e-10)
        for tol in targets:
            (x, ri), ms = _timed(lambda: rka.refine_solve(
                None, b, plan=PA, plan_t=PT, q=q, alpha=al, accumulate=acc, inner_iters=k_in,
                range_iters=k_col, range_q=qc, range_alpha=alc, max_sweeps=8, tol=tol,
                x_ref=x_ls, raise_on_error=False))
            entry[f"to_{tol:g}"] = {"ms": ms, "sweeps": ri.sweeps, "status": ri.status,
                                    "per_sweep_rel_err": ri.measures,
                                    "final_rel_err": float((x - x_ls).norm() / x_ls.norm()),
                                    "projections": ri.projections}
            if ri.status < 0 and ri.status != rka.NOT_CONVERGED:
                entry[f"to_{tol:g}"]["error"] = rka.lib().rka_last_error().decode()
        runs[name] = entry
        PA.close()
        PT.close()
        del At, b, x_ls
        if As is not A64:
            del As
        torch.cuda.empty_cache()
    for name in ("bf16", "fp32"):
        runs[name]["speedup_vs_fp64_to_1e-06"] = (runs["fp64"]["to_1e-06"]["ms"] /
                                                 runs[name]["to_1e-06"]["ms"])
    out["runs"] = runs
    del A64, xs, e
    torch.cuda.empty_cache()
    return out


def bench_batching(rka, workloads, count, n_sample, seed):
    """512 FP32 systems (m, n log-uniform, m >= 4n, rows scaled log-uniform in
    [0.1, 10], planted x*) plus a 50000 x 2000 matrix with 64 planted
    right-hand sides, to 1e-6 relative error in graph-captured batch solves
    (binary32, with FP64 refinement sweeps for the systems whose binary32
    iteration stalls above 1e-6);
    against plain FP64 RKA (q = 16, alpha = 1) solving a random sample of the
    same systems one by one, extrapolated by system count."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    shapes = workloads.batch_shapes(count, seed=workloads.DATA_SEED + 4)
    gen = torch.Generator(device=dev)
    gen.manual_seed(workloads.DATA_SEED + 5)
    systems, planted = [], []
    total_bytes = 0
    for (m, n) in shapes:
        A = torch.randn((m, n), generator=gen, device=dev, dtype=torch.float32)
        sc = torch.exp(torch.empty(m, device=dev, dtype=torch.float64).uniform_(
            math.log(0.1), math.log(10.0), generator=gen))
        A *= sc.to(torch.float32)[:, None]
        xs = torch.randn(n, generator=gen, device=dev, dtype=torch.float64)
        b = A.to(torch.float64) @ xs
        systems.append(rka.BatchSystem(A=A, B=b, X=torch.zeros(n, dtype=torch.float64,
                                                               device=dev),
                                       X_ref=xs, alpha=0.0, max_iter=60000))
        planted.append(xs)
        total_bytes += m * n * 4
    Msh, Nsh, R = 50000, 2000, 64
    Ash = torch.randn((Msh, Nsh), generator=gen, device=dev, dtype=torch.float32)
    Xs = torch.randn((R, Nsh), generator=gen, device=dev, dtype=torch.float64)
    Bsh = Xs @ Ash.to(torch.float64).T
    systems.append(rka.BatchSystem(A=Ash, B=Bsh.contiguous(),
                                   X=torch.zeros((R, Nsh), dtype=torch.float64, device=dev),
                                   X_ref=Xs, alpha=0.0, max_iter=60000))
    total_bytes += Msh * Nsh * 4
    torch.cuda.synchronize()
    trials, tune_ms = _timed(lambda: rka.batch_tune(systems, seed=seed))
    # iteration caps as a budget of 4e6 dependent projection steps per worker
    # (an iteration is block_size steps plus the average)
    for S in systems:
        S.max_iter = int(4e6 // (S.block_size + 2))
    (res, st), ms = _timed(lambda: rka.batch_solve(systems, seed=seed, tol=1e-6, check_every=10,
                                                   graph=True, refine_sweeps=3,
                                                   raise_on_error=False))
    ok = sum(1 for r in res if r["status"] == 0)
    classes = {}
    for r, S in zip(res, systems):
        n = S.A.shape[1]
        c = 1 << max(0, (n - 1).bit_length())
        key = f"n<={c}"
        e = classes.setdefault(key, {"systems": 0, "params": set(), "not_converged": 0,
                                     "max_iterations": 0})
        e["systems"] += 1
        e["params"].add((r["tpr"], r["q"], r["block_size"], round(r["alpha"], 3),
                         r["rhs_per_task"]))
        e["max_iterations"] = max(e["max_iterations"], r["iterations"])
        if r["status"] != 0:
            e["not_converged"] += 1
    for e in classes.values():
        e["params"] = sorted(e["params"])
    unconv = [{"m": S.A.shape[0], "n": S.A.shape[1], "iterations": r["iterations"],
               "rel": r["rel"], "tpr": r["tpr"], "q": r["q"], "bs": r["block_size"]}
              for r, S in zip(res, systems) if r["status"] != 0][:12]
    proj = sum(r["iterations"] * r["q"] * r["block_size"] * S.B.shape[0] if S.B.dim() > 1
               else r["iterations"] * r["q"] * r["block_size"] for r, S in zip(res, systems))
    worst = max(r["rel"] for r in res)
    # plain FP64 RKA on a sample, one system at a time, stratified by how much
    # work the batch needed (row bytes to convergence): the hardest 5 % form
    # one stratum, the rest another; each stratum's mean time is scaled by its
    # size
    rng = np.random.default_rng(seed)
    work = np.array([r["iterations"] * r["q"] * r["block_size"] * S.A.shape[1]
                     for r, S in zip(res[:count], systems[:count])], dtype=np.float64)
    order = np.argsort(-work)
    n_hard = max(1, count // 20)
    hard, rest = order[:n_hard], order[n_hard:]
    k_hard = min(len(hard), max(1, n_sample // 4))
    k_rest = min(len(rest), max(1, n_sample - k_hard))
    strata = [(rng.choice(hard, size=k_hard, replace=False), len(hard)),
              (rng.choice(rest, size=k_rest, replace=False), len(rest))]
    t_plain = 0.0
    extrap = 0.0
    extrap_tuned = 0.0
    plain = []

    def tuned_alpha(A64, qq):
        lo, hi, F = rka.spectral_bounds(A64, steps=min(120, min(A64.shape)), seed=5)
        return rka.alpha_star(lo / F, hi / F, qq)

    for members, size in strata:
        t_stratum = t_tuned = 0.0
        for i in sorted(int(v) for v in members):
            S = systems[i]
            A64 = S.A.to(torch.float64)
            (x, info, _), t = _timed(lambda: rka.solve_ex(A64, S.B, method=0, q=16, alpha=1.0,
                                                          max_iter=2000000, tol=1e-6,
                                                          x_ref=planted[i], check_every=10,
                                                          raise_on_error=False))
            # tuned plain FP64: q = 64 (at most m / 4) with alpha* of Eq. (6)
            qt = max(1, min(64, S.A.shape[0] // 4))
            at, t_alpha = _timed(lambda: tuned_alpha(A64, qt))
            (x, info_t, _), tt = _timed(lambda: rka.solve_ex(A64, S.B, method=0, q=qt, alpha=at,
                                                             max_iter=2000000, tol=1e-6,
                                                             x_ref=planted[i], check_every=10,
                                                             raise_on_error=False))
            t_stratum += t
            t_tuned += tt
            plain.append({"m": S.A.shape[0], "n": S.A.shape[1], "ms": t,
                          "iterations": info.iterations, "status": info.status,
                          "tuned_q": qt, "tuned_alpha": at, "tuned_ms": tt,
                          "tuned_alpha_ms": t_alpha, "tuned_iterations": info_t.iterations,
                          "tuned_status": info_t.status,
                          "stratum": "hardest 5%" if size == len(hard) else "rest"})
            del A64
        t_plain += t_stratum
        extrap += t_stratum / len(members) * size
        extrap_tuned += t_tuned / len(members) * size
    A64 = Ash.to(torch.float64)
    t_sh = t_sh_tuned = 0.0
    a_sh = tuned_alpha(A64, 64)
    for r in range(4):
        (x, info, _), t = _timed(lambda: rka.solve_ex(A64, Bsh[r].contiguous(), method=0, q=16,
                                                      alpha=1.0, max_iter=2000000, tol=1e-6,
                                                      x_ref=Xs[r].contiguous(), check_every=10,
                                                      raise_on_error=False))
        (x, info, _), tt = _timed(lambda: rka.solve_ex(A64, Bsh[r].contiguous(), method=0, q=64,
                                                       alpha=a_sh, max_iter=2000000, tol=1e-6,
                                                       x_ref=Xs[r].contiguous(), check_every=10,
                                                       raise_on_error=False))
        t_sh += t
        t_sh_tuned += tt
    del A64
    extrap += t_sh / 4 * R
    extrap_tuned += t_sh_tuned / 4 * R
    # HBM bytes of the batch: the rows each task read (once per iteration,
    # worker and projection, shared by the task's right-hand sides) plus one
    # FP64-residual pass over every matrix per refinement sweep
    row_bytes = 0
    for r, S in zip(res, systems):
        n_ = S.A.shape[1]
        nrhs = S.B.shape[0] if S.B.dim() > 1 else 1
        tasks = -(-nrhs // max(1, r["rhs_per_task"]))
        row_bytes += r["iterations"] * r["q"] * r["block_size"] * (4 * n_ + 20) * tasks
    resid_bytes = 3 * total_bytes
    return {
        "systems": count, "shared_matrix": f"{Msh}x{Nsh} with {R} right-hand sides",
        "matrix_bytes": total_bytes, "tune_ms": tune_ms, "tune_trials": trials,
        "batch_ms_to_1e-6": ms, "graph_ms": st["iterate_ms"], "tasks": st["tasks"],
        "chunks": st["chunks"], "converged_systems": ok, "worst_rel_err": worst,
        "projections_upper_bound": proj, "classes": classes, "not_converged_sample": unconv,
        "plain_fp64_rka_sample": plain, "plain_fp64_shared_ms_per_rhs": t_sh / 4,
        "plain_fp64_extrapolated_ms": extrap,
        "speedup_vs_plain_fp64": extrap / ms,
        "plain_fp64_tuned_extrapolated_ms": extrap_tuned,
        "speedup_vs_tuned_plain_fp64": extrap_tuned / ms,
        "hbm_bytes_upper_bound": row_bytes + resid_bytes,
        "hbm_gbps": (row_bytes + resid_bytes) / (ms / 1e3) / 1e9,
        "hbm_frac_of_peak": (row_bytes + resid_bytes) / (ms / 1e3) / 1e9 / PEAK_HBM_GBPS,
        "hbm_note": ("rows read per task iteration (iterations summed over the refinement "
                     "sweeps; an upper bound, since stopped tasks read no rows) plus one FP32 "
                     "pass per matrix per sweep for the FP64 residual, over the graph time "
                     "including set-up"),
        "note": ("plain FP64 RKA measured one solve at a time -- q=16, alpha=1, and tuned: "
                 "q=64 (at most m/4) with alpha* from the device Lanczos (its time excluded) -- "
                 "on a sample "
                 f"stratified by the batch's work to convergence ({k_hard} of the hardest "
                 f"{len(hard)} systems, {k_rest} of the other {len(rest)}) and on 4 of the "
                 "shared right-hand sides; each stratum's mean scaled by its size"),
    }


def bench_differentiation(rka):
    """Forward + backward of the differentiable solve on a 20000 x 1000 system
    (FP32 storage) against the same with FP64 storage; accuracy against an
    FP64 normal-equations reference computed on the GPU."""
    import torch
    from paper_2401_17474_amd.autograd import SolveOpts, lsq_solve
    dev = torch.device("cuda:0")
    m, n, q = 20000, 1000, 64
    gen = torch.Generator(device=dev)
    gen.manual_seed(240117474 + 6)
    A64 = torch.randn((m, n), generator=gen, device=dev, dtype=torch.float64)
    A32 = A64.to(torch.float32)
    A64 = A32.to(torch.float64)  # the problem matrix is the FP32 one
    xs = torch.randn(n, generator=gen, device=dev, dtype=torch.float64)
    b = A64 @ xs + 0.1 * torch.randn(m, generator=gen, device=dev, dtype=torch.float64)
    t = torch.randn(n, generator=gen, device=dev, dtype=torch.float64)
    G = A64.T @ A64
    ev = torch.linalg.eigvalsh(G)
    F = float(torch.trace(G))
    s_ext = (float(ev[0]) / F, float(ev[-1]) / F)
    al = rka.alpha_star(*s_ext, q)
    k = int(math.ceil(1.1 * 9.2 / _rate(s_ext, al, q)))
    # reference: x_LS and the gradient of L = ||x - t||^2 from the normal equations
    L = torch.linalg.cholesky(G)
    x_ref = torch.cholesky_solve((A64.T @ b)[:, None], L)[:, 0]
    g = 2 * (x_ref - t)
    lam = torch.cholesky_solve(g[:, None], L)[:, 0]
    z = A64 @ lam
    r = b - A64 @ x_ref
    dA_ref = torch.outer(r, lam) - torch.outer(z, x_ref)
    out = {"shape": f"{m}x{n}", "q": q, "alpha": al, "inner_iters": k, "sweeps": 3}
    for name, A in (("fp32", A32), ("fp64", A64)):
        opts = SolveOpts(q=q, alpha=al, inner_iters=k, range_iters=k, sweeps=3,
                         accumulate=1 if name == "fp32" else 0, seed=3)
        times = []
        for rep in range(3):
            Ad = A.detach().clone().requires_grad_(True)
            bd = b.detach().clone().requires_grad_(True)

            def fb():
                x = lsq_solve(Ad, bd, opts)
                torch.sum((x - t) ** 2).backward()
                return x
            x, ms = _timed(fb)
            times.append(ms)
        times.sort()
        out[name] = {
            "forward_backward_ms": times[1],
            "rel_err_x": float((x - x_ref).norm() / x_ref.norm()),
            "rel_err_dA": float((Ad.grad.to(torch.float64) - dA_ref).norm() / dA_ref.norm()),
            "rel_err_db": float((bd.grad - z).norm() / z.norm()),
        }
    out["speedup_fp32_vs_fp64"] = out["fp64"]["forward_backward_ms"] / out["fp32"][
        "forward_backward_ms"]
    return out


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    counter runs (profiles/pmc_traffic.json, scaled by a copy of known size),
    or None when the counters were not taken on this kernel or were taken on
    other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        for e in d["entries"]:
            if e.get("kernel") != kernel:
                continue
            h = hashlib.sha256()
            for p in e["sources"]:
                with open(os.path.join(ROOT, p), "rb") as f:
                    h.update(f.read())
            if h.hexdigest() == e.get("sources_sha256"):
                return e["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError, TypeError):
        return None
    return None


def bench_distributed(rka, workloads):
    """The four sampling / weight variants of Sec. 3.3.2 (Table 1's layout):
    outer iterations of RKA to 1e-8 relative error on a planted 10000 x 2500
    system (Table 1's 4:1 shape), q in {2, 4, 8, 16}; full-matrix alpha* from
    the device Lanczos, partial-matrix alpha per worker block."""
    import torch
    dev = torch.device("cuda:0")
    m, n = 10000, 2500
    A, xs, b = workloads.gaussian_system(m, n, seed=workloads.DATA_SEED + 7, rng="torch",
                                         device=dev)
    lo, hi, F = rka.spectral_bounds(A, steps=120, seed=5)
    out = {"shape": f"{m}x{n}", "tol": 1e-8, "rows": []}
    for q in (2, 4, 8, 16):
        a_full = rka.alpha_star(lo / F, hi / F, q)
        wa, pa_ms = _timed(lambda: rka.partial_alpha(A, q, steps=120, seed=9))
        row = {"q": q, "alpha_full": a_full,
               "alpha_partial_range": [float(wa.min()), float(wa.max())],
               "partial_alpha_ms": pa_ms}
        for name, sampling, walpha in (("full_access_full_alpha", 0, None),
                                       ("distributed_full_alpha", 1, None),
                                       ("full_access_partial_alpha", 0, wa),
                                       ("distributed_partial_alpha", 1, wa)):
            (x, info, st), ms = _timed(lambda: rka.solve_ex(
                A, b, method=0, q=q, alpha=a_full, max_iter=2000000, tol=1e-8, x_ref=xs,
                check_every=10, seed=3, sampling=sampling, worker_alpha=walpha,
                raise_on_error=False))
            row[name] = {"iterations": info.iterations, "status": info.status, "ms": ms}
        out["rows"].append(row)
    return out


def bench_coherent(rka, workloads):
    """Row order on the coherent-row set of Sec. 3.1 (20000 x 1000, every row
    with its own mean and spread): time and iterations to 1e-6 relative error
    of Cyclic Kaczmarz (Sec. 2.1) with the rows as drawn and with the same
    rows sorted so that neighbours are nearly parallel, against RK and RKA
    sampling by row norm, with alpha = 1 and with alpha* of Eq. (6) (the
    second case of Eq. (6) at q = 64 on this set)."""
    import torch
    dev = torch.device("cuda:0")
    m, n, tol, cap = 20000, 1000, 1e-6, 1000000
    out = {"shape": f"{m}x{n}", "tol": tol, "max_iter": cap, "runs": []}
    for order in ("drawn", "coherent"):
        Ah, xh, bh = workloads.paper_rows_system(m, n, seed=workloads.DATA_SEED + 11, order=order)
        A = torch.from_numpy(Ah).to(dev)
        b = torch.from_numpy(bh).to(dev)
        xs = torch.from_numpy(xh).to(dev)
        del Ah
        lo, hi, F = rka.spectral_bounds(A, steps=150, seed=5)
        s_min, s_max = lo / F, hi / F
        out.setdefault("s_min", s_min)
        out.setdefault("s_max", s_max)
        a64 = rka.alpha_star(s_min, s_max, 64)
        out["alpha_star_q64"] = a64
        out["alpha_star_q64_case"] = 1 if s_max - s_min <= 1.0 / 63 else 2
        runs = [("cyclic_kaczmarz", 1, 1.0, 2), ("rk", 1, 1.0, 0), ("rka_q64_alpha1", 64, 1.0, 0),
                ("rka_q64_alpha_star", 64, a64, 0), ("cyclic_q64_alpha_star", 64, a64, 2)]
        for name, q, alpha, sampling in runs:
            (x, info, st), ms = _timed(lambda: rka.solve_ex(
                A, b, method=0, q=q, alpha=alpha, max_iter=cap, tol=tol, x_ref=xs,
                check_every=50, seed=3, sampling=sampling, raise_on_error=False))
            out["runs"].append({"order": order, "name": name, "q": q, "alpha": alpha,
                                "sampling": ["by_norm", "blocks", "cyclic"][sampling],
                                "iterations": info.iterations, "projections": info.projections,
                                "rel_err": info.rel_err, "status": info.status, "ms": ms})
        del A, b, xs
        torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the solver "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nbytes}), flush=True)
        return

    import paper_2401_17474_amd as rka
    import workloads

    if not os.path.exists(rka.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    rka.lib()
    dev = torch.device("cuda:0")
    m, n = args.m, args.n
    log(f"[bench] generating {m}x{n} FP64 system on {torch.cuda.get_device_name(0)}")
    A, xs, b = workloads.gaussian_system(m, n, seed=workloads.DATA_SEED + 2, noise_var=1e-2,
                                         rng="torch", device=dev)
    torch.cuda.synchronize()

    # least-squares reference (normal equations, well conditioned here, plus one
    # refinement step -- a measurement aid) and alpha*(q) from the extreme
    # singular values
    log("[bench] least-squares reference and alpha*")
    G = A.T @ A
    L = torch.linalg.cholesky(G)
    x_ls = torch.cholesky_solve((A.T @ b)[:, None], L)[:, 0]
    r = b - A @ x_ls
    x_ls = x_ls + torch.cholesky_solve((A.T @ r)[:, None], L)[:, 0]
    # alpha* (Eq. (6)) from the extreme eigenvalues of A^T A, on the device
    (lmin, lmax, F), astar_ms = _timed(lambda: rka.spectral_bounds(A, steps=160, seed=7))
    s_min, s_max = lmin / F, lmax / F
    astar = {q: rka.alpha_star(s_min, s_max, q) for q in (16, 64, 256)}
    del G, L, r
    torch.cuda.empty_cache()

    log("[bench] copy ceiling")
    ceiling = copy_ceiling()
    cells = make_cells(args.cells, astar)
    esz = 8
    bytes_per_proj = n * esz + 8 + 8 + 4  # row + b_i + ||a_i||^2 + index
    out = torch.empty(n, dtype=torch.float64, device=dev)
    # the sampling distribution of Eq. (4), once per matrix: every cell's
    # solve reuses its row norms and running sum
    plan, plan_ms = _timed(lambda: rka.Plan(A))

    def run_cell(c, seed):
        meth, q, bs, alpha, _ = c
        K = max(1, args.rows_per_cell // (q * bs))
        x, info, st = plan.solve(b, method=0 if meth == "rka" else 1, q=q, block_size=bs,
                                 alpha=alpha, max_iter=K, seed=seed, timing=True, out=out)
        return x, info, st

    log(f"[bench] warmup {args.warmup} step(s) of {len(cells)} cells")
    for w in range(args.warmup):
        for c in cells:
            run_cell(c, args.seed + 1000 + w)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} step(s)")
    per_cell = {i: {"proj": 0, "wall": 0.0, "iter_ms": 0.0, "coef_ms": 0.0, "launches": 0,
                    "setup_ms": 0.0, "sample_ms": 0.0} for i in range(len(cells))}
    kern = {}
    errs = {}
    total_proj = 0
    step_s = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        t_step = time.perf_counter()
        for i, c in enumerate(cells):
            t0 = time.perf_counter()
            x, info, st = run_cell(c, args.seed + s)
            dt = time.perf_counter() - t0
            pc = per_cell[i]
            pc["proj"] += info.projections
            pc["wall"] += dt
            pc["iter_ms"] += st["iterate_ms"]
            pc["coef_ms"] += st["coef_ms"]
            pc["launches"] += st["iterate_launches"]
            pc["setup_ms"] += st["norms_ms"] + st["prefix_ms"]
            pc["sample_ms"] += st["sample_ms"]
            pc["stats"] = st
            total_proj += info.projections
            name = kernel_name(st, rkab=c[0] == "rkab", bs=c[2])
            kk = kern.setdefault(name, {"ms": 0.0, "launches": 0, "bytes": 0.0})
            kk["ms"] += st["iterate_ms"]
            kk["launches"] += st["iterate_launches"]
            kk["bytes"] += info.projections * bytes_per_proj
            if st["kernel"] == 4 and st["coef_ms"] > 0:
                # the coefficient pass streams every row of the chunk once
                cname = "blk_coef_rkab_kernel<double>" if c[0] == "rkab" else "blk_coef_kernel<double>"
                kc = kern.setdefault(cname, {"ms": 0.0, "launches": 0, "bytes": 0.0})
                kc["ms"] += st["coef_ms"]
                kc["launches"] += st["iterate_launches"]
                kc["bytes"] += info.projections * n * esz
            if s == args.steps - 1:
                errs[i] = float((x - x_ls).norm() / x_ls.norm())
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t_step)
        log(f"[bench] step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    # every step moves the same projections: the headline is the median step
    proj_per_step = total_proj / args.steps
    med_step = sorted(step_s)[len(step_s) // 2]
    value = proj_per_step / med_step
    cells_out = []
    for i, c in enumerate(cells):
        pc = per_cell[i]
        meth, q, bs, alpha, alab = c
        it_s = (pc["iter_ms"] + pc["coef_ms"]) / 1e3
        cells_out.append({
            "method": meth, "q": q, "block_size": bs, "alpha": round(alpha, 4), "alpha_kind": alab,
            "projections_per_s": pc["proj"] / pc["wall"],
            "kernel_projections_per_s": pc["proj"] / it_s if it_s > 0 else None,
            "kernel_hbm_gbps": pc["proj"] * bytes_per_proj / it_s / 1e9 if it_s > 0 else None,
            "iterate_ms_per_solve": pc["iter_ms"] / args.steps,
            "coef_ms_per_solve": pc["coef_ms"] / args.steps,
            "setup_ms_per_solve": pc["setup_ms"] / args.steps,
            "sample_ms_per_solve": pc["sample_ms"] / args.steps,
            "kernel": kernel_name(pc["stats"], rkab=meth == "rkab", bs=bs), "grid": pc["stats"]["grid"],
            "threads": pc["stats"]["threads"],
            "rel_err_vs_x_ls": errs.get(i),
        })
    dom_name, dom = max(kern.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": pmc_traffic(dom_name),
            "kernel": dom_name, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch":
            bytes_per_launch, "bytes_per_projection": bytes_per_proj,
            "copy_ceiling_gbps": round(ceiling["gbps"], 1),
            "frac_of_copy_ceiling": round(achieved / ceiling["gbps"], 4)}

    # time to the error plateau of every cell (two passes, Sec. 3.1)
    plateau = []
    if not args.no_plateau:
        s_ext = (s_min, s_max)
        for c in cells:
            meth, q, bs, alpha, alab = c
            log(f"[bench] time to plateau {meth} q={q} bs={bs} alpha={alab}")
            rate = _rate(s_ext, alpha if meth == "rka" else 1.0, q)
            r = time_to_plateau(plan, b, x_ls, c, rate, seed=args.seed + 77)
            r.update({"method": meth, "q": q, "block_size": bs, "alpha_kind": alab})
            plateau.append(r)

    forms = {}
    if not args.no_forms:
        wanted = set(args.forms.split(","))
        for name, fn in (("precision", lambda: bench_precision(rka, A, xs, b, x_ls,
                                                                (s_min, s_max))),
                         ("precision_200000x20000", lambda: bench_precision_large(rka)),
                         ("batching", lambda: bench_batching(rka, workloads, args.batch_systems,
                                                             args.batch_sample, args.seed)),
                         ("differentiation", lambda: bench_differentiation(rka)),
                         ("distributed_approach", lambda: bench_distributed(rka, workloads)),
                         ("coherent_rows", lambda: bench_coherent(rka, workloads))):
            if name not in wanted:
                continue
            log(f"[bench] form: {name}")
            try:
                forms[name] = fn()
            except Exception as e:  # a failing form must not hide the main line
                forms[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
            log(f"[bench] form {name} done")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        Ah = A.cpu().numpy()
        bh = b.cpu().numpy()
        cpu = cpu_baseline(Ah, bh, args.cpu_seconds)
        del Ah
        log("[bench] CPU oracle on the smaller configurations")
        cpu["other_configurations"] = cpu_baseline_cells(workloads)

    line = {
        "metric": METRIC, "value": value, "unit": "row projections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": med_step * 1e3,
        "mean_ms_per_step": wall / args.steps * 1e3, "value_mean": total_proj / wall,
        "step_ms": [round(t * 1e3, 2) for t in step_s],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RKA/RKAB grid on a {m}x{n} FP64 N(0,1) system, "
                               "b = A x* + N(0, 1e-2)",
                   "m": m, "n": n, "rows_per_cell": args.rows_per_cell,
                   "cells": len(cells), "parallelism": "single GPU"},
        "hbm_gbps": value * bytes_per_proj / 1e9,
        "roofline": roof,
        "copy_ceiling": ceiling,
        "plan_setup_ms": plan_ms,
        "time_to_plateau": plateau,
        "cpu_baseline": cpu,
        "alpha_star": {str(q): astar[q] for q in astar}, "s_min": s_min, "s_max": s_max,
        "alpha_star_device_ms": astar_ms,
        "cells": cells_out,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
