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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=80000)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--rows-per-cell", type=int, default=819200)
    ap.add_argument("--cells", default="all", help="all | rka | rkab | comma list like rkab:256:10")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def lanczos_extremes(G, steps=160):
    """Extreme eigenvalues of the SPD matrix G (torch, FP64) by Lanczos with
    full reorthogonalization; used only to set alpha* (Eq. (6))."""
    import numpy as np
    import torch
    n = G.shape[0]
    gen = torch.Generator(device=G.device)
    gen.manual_seed(7)
    v = torch.randn(n, generator=gen, device=G.device, dtype=torch.float64)
    v /= v.norm()
    V = torch.zeros((steps, n), device=G.device, dtype=torch.float64)
    al, be = [], []
    b_prev = 0.0
    v_prev = torch.zeros_like(v)
    for j in range(steps):
        V[j] = v
        w = G @ v - b_prev * v_prev
        a = float(w @ v)
        w -= a * v
        w -= V[: j + 1].T @ (V[: j + 1] @ w)
        b = float(w.norm())
        al.append(a)
        be.append(b)
        if b < 1e-12:
            break
        v_prev, v, b_prev = v, w / b, b
    k = len(al)
    T = np.diag(al) + np.diag(be[: k - 1], 1) + np.diag(be[: k - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


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


def kernel_name(stats):
    # template instance as named in the library (double storage, 16-byte vecs)
    if stats["kernel"] == 1:
        return f"rka_col_kernel<double, 2, {stats['bucket']}>"
    return f"rkab_kernel<double, 2, {stats['bucket']}>"


def cpu_baseline(A, b, seconds):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    q = 16

    def timed(K):
        t0 = time.perf_counter()
        _, info = oracle.rka(A, b, q=q, alpha=1.0, max_iter=K, seed=3)
        return time.perf_counter() - t0, info

    t_setup, _ = timed(0)          # row norms + running sum over all of A
    t_probe, _ = timed(40)
    per_iter = max((t_probe - t_setup) / 40, 1e-6)
    K = max(40, int((seconds - t_setup) / per_iter))
    dt, info = timed(K)
    return {"value": info["projections"] / dt, "unit": "row projections/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"oracle RKA (plain C, FP64, single thread) on the same {A.shape[0]}x"
                       f"{A.shape[1]} FP64 system, q={q}, alpha=1, {K} iterations "
                       f"({info['projections']} projections) including its row norms and "
                       f"running sum, {dt:.1f} s wall"),
            "host_cpu": _cpu_model(), "host_threads": os.cpu_count()}


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
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): this build "
              "has no multi-GPU path; how it would shard is described in DESIGN.md.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

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
    # refinement step) and alpha*(q) from the extreme singular values
    log("[bench] least-squares reference and alpha*")
    G = A.T @ A
    L = torch.linalg.cholesky(G)
    x_ls = torch.cholesky_solve((A.T @ b)[:, None], L)[:, 0]
    r = b - A @ x_ls
    x_ls = x_ls + torch.cholesky_solve((A.T @ r)[:, None], L)[:, 0]
    F = float((A * A).sum())
    lmin, lmax = lanczos_extremes(G)
    s_min, s_max = lmin / F, lmax / F
    astar = {q: rka.alpha_star(s_min, s_max, q) for q in (16, 64, 256)}
    del G, L, r
    torch.cuda.empty_cache()

    cells = make_cells(args.cells, astar)
    esz = 8
    bytes_per_proj = n * esz + 8 + 8 + 4  # row + b_i + ||a_i||^2 + index
    out = torch.empty(n, dtype=torch.float64, device=dev)

    def run_cell(c, seed):
        meth, q, bs, alpha, _ = c
        K = max(1, args.rows_per_cell // (q * bs))
        x, info, st = rka.solve_ex(A, b, method=0 if meth == "rka" else 1, q=q, block_size=bs,
                                   alpha=alpha, max_iter=K, seed=seed, timing=True, out=out)
        return x, info, st

    log(f"[bench] warmup {args.warmup} step(s) of {len(cells)} cells")
    for w in range(args.warmup):
        for c in cells:
            run_cell(c, args.seed + 1000 + w)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} step(s)")
    per_cell = {i: {"proj": 0, "wall": 0.0, "iter_ms": 0.0, "launches": 0, "setup_ms": 0.0,
                    "sample_ms": 0.0} for i in range(len(cells))}
    kern = {}
    errs = {}
    total_proj = 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        for i, c in enumerate(cells):
            t0 = time.perf_counter()
            x, info, st = run_cell(c, args.seed + s)
            dt = time.perf_counter() - t0
            pc = per_cell[i]
            pc["proj"] += info.projections
            pc["wall"] += dt
            pc["iter_ms"] += st["iterate_ms"]
            pc["launches"] += st["iterate_launches"]
            pc["setup_ms"] += st["norms_ms"] + st["prefix_ms"]
            pc["sample_ms"] += st["sample_ms"]
            pc["stats"] = st
            total_proj += info.projections
            name = kernel_name(st)
            kk = kern.setdefault(name, {"ms": 0.0, "launches": 0, "bytes": 0.0})
            kk["ms"] += st["iterate_ms"]
            kk["launches"] += st["iterate_launches"]
            kk["bytes"] += info.projections * bytes_per_proj
            if s == args.steps - 1:
                errs[i] = float((x - x_ls).norm() / x_ls.norm())
        log(f"[bench] step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    value = total_proj / wall
    cells_out = []
    for i, c in enumerate(cells):
        pc = per_cell[i]
        meth, q, bs, alpha, alab = c
        it_s = pc["iter_ms"] / 1e3
        cells_out.append({
            "method": meth, "q": q, "block_size": bs, "alpha": round(alpha, 4), "alpha_kind": alab,
            "projections_per_s": pc["proj"] / pc["wall"],
            "kernel_projections_per_s": pc["proj"] / it_s if it_s > 0 else None,
            "kernel_hbm_gbps": pc["proj"] * bytes_per_proj / it_s / 1e9 if it_s > 0 else None,
            "iterate_ms_per_solve": pc["iter_ms"] / args.steps,
            "setup_ms_per_solve": pc["setup_ms"] / args.steps,
            "sample_ms_per_solve": pc["sample_ms"] / args.steps,
            "kernel": kernel_name(pc["stats"]), "grid": pc["stats"]["grid"],
            "threads": pc["stats"]["threads"],
            "rel_err_vs_x_ls": errs.get(i),
        })
    dom_name, dom = max(kern.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None,
            "kernel": dom_name, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch":
            bytes_per_launch, "bytes_per_projection": bytes_per_proj}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        Ah = A.cpu().numpy()
        bh = b.cpu().numpy()
        cpu = cpu_baseline(Ah, bh, args.cpu_seconds)
        del Ah

    line = {
        "metric": METRIC, "value": value, "unit": "row projections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RKA/RKAB grid on a {m}x{n} FP64 N(0,1) system, "
                               "b = A x* + N(0, 1e-2)",
                   "m": m, "n": n, "rows_per_cell": args.rows_per_cell,
                   "cells": len(cells), "parallelism": "single GPU"},
        "hbm_gbps": value * bytes_per_proj / 1e9,
        "roofline": roof,
        "cpu_baseline": cpu,
        "alpha_star": {str(q): astar[q] for q in astar}, "s_min": s_min, "s_max": s_max,
        "cells": cells_out,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
