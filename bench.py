"""Benchmark: unit-cell Stokes permeability on one MI355X.

Workload (one "step"): the 3D Stokes cell problem on a 128^3 periodic cell of
randomly placed overlapping spheres (radius 8 voxels, centres from SplitMix64
seed 1, added until the pore fraction first drops to 0.40), solved by the ADMM
of Section 3.1 for the three unit pressure gradients e_x, e_y, e_z to
eps = 1e-6 (FP32 fields and transforms, FP64 reductions), followed by the full
permeability tensor (eq. K).  Inputs are resident in HBM before timing starts.

Prints ONE JSON line.  Throughput = voxel-iterations per second over the timed
steps.  The roofline object covers the kernel with the largest share of time in
a profiled solve (HIP events on the library stream); cpu_baseline times the
FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="cell side (voxels)")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle iterations in the CPU sample")
    return ap.parse_args()


def kernel_bytes(kind: str, n: int, d: int, nsolid: int, real_bytes: int = 4) -> float:
    """Algorithmic HBM bytes one launch of `kind` must move (FP32 fields).
    Half spectra hold nspec = n*n*(n/2+1) complex values per field."""
    ntot = n ** d
    nspec = (n ** (d - 1)) * (n // 2 + 1)
    cb = 2 * real_bytes
    if kind == "green":   # d spectral fields in+out, q-hat and div-hat in+out
        return nspec * cb * (2 * d + 4)
    if kind in ("y_inv", "y_fwd"):
        return nspec * cb * 2 * d
    if kind == "local":   # spectra in; u in+out; a in+out on solid voxels; H
        return d * nspec * cb + 2 * d * ntot * real_bytes + 2 * d * nsolid * real_bytes + ntot
    if kind == "rhs":     # u in; a in on solid voxels; H; spectra out
        return d * ntot * real_bytes + d * nsolid * real_bytes + ntot + d * nspec * cb
    return float("nan")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent cells or directions would shard one per GPU, see DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2312_15554_amd import inputs as I
    from paper_2312_15554_amd.api import acm_effective_props, acm_stokes_solve

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    n, d = args.n, 3
    H_np = I.overlapping_spheres(n, 8.0 * n / 128.0, 0.40, seed=1)
    nsolid = int(H_np.sum())
    porosity = 1.0 - nsolid / H_np.size
    H = torch.from_numpy(H_np).cuda()
    dirs = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)]
    us = [torch.empty((d, n, n, n), dtype=torch.float32, device="cuda") for _ in dirs]
    pen = dict(tau=(5.0, 10.0, 5.0))  # random-geometry schedule (Section 4.1 footnote)

    def step():
        its, secs = [], []
        for g, u in zip(dirs, us):
            r = acm_stokes_solve(H, g, penalty=pen, eps=args.eps, max_iter=200000, u=u,
                                 want_q=False)
            its.append(r["stats"]["iters"])
            secs.append(r["stats"]["seconds"])
            if not r["stats"]["converged"]:
                raise RuntimeError(f"solve did not converge: {r['stats']}")
        K = acm_effective_props(H, us, nu=1.0)["K"]
        return its, secs, K

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        its_w, secs_w, _ = step()
        log(f"warmup {w}: iterations {its_w}, seconds {[round(x, 3) for x in secs_w]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step())
        log(f"step {k}: iterations {results[-1][0]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_vi = sum(sum(r[0]) for r in results) * float(n ** d)
    wall = t1 - t0
    its, secs, K = results[-1]

    # ---- roofline: profiled solve (eager launches, HIP events per kernel)
    rp = acm_stokes_solve(H, dirs[0], penalty=pen, eps=args.eps, max_iter=200000, u=us[0],
                          want_q=False, profile=True)
    km, kc = rp["stats"]["kernel_ms"], rp["stats"]["kernel_calls"]
    share = {k: km[k] for k in km if kc[k] > 0}
    dom = max(share, key=share.get)
    avg_s = km[dom] / kc[dom] * 1e-3
    algo = kernel_bytes(dom, n, d, nsolid)
    achieved = algo / avg_s / 1e9
    per_kernel = {k: dict(avg_us=round(km[k] / kc[k] * 1e3, 2), calls=kc[k],
                          GBps=round(kernel_bytes(k, n, d, nsolid) / (km[k] / kc[k] * 1e-3) / 1e9, 1))
                  for k in share}
    iter_us_profiled = 1e3 * sum(km.values()) / max(1, rp["stats"]["iters"])

    log(f"profiled solve: dominant kernel {dom}, {per_kernel}")
    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same cell
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle sample")
        from oracle import acm_oracle as O
        threads = max(1, min(os.cpu_count() or 1, 16))
        O.set_workers(threads)
        tc0 = time.perf_counter()
        O.stokes_admm(H_np, dirs[0], tau=(5.0, 10.0, 5.0), eps=0.0, max_iter=args.cpu_iters)
        tc1 = time.perf_counter()
        cpu = dict(value=args.cpu_iters * float(n ** d) / (tc1 - tc0), unit="voxel-iters/s",
                   cores=threads, kind="oracle",
                   sample=f"{args.cpu_iters} ADMM iterations of the FP64 oracle on the same "
                          f"{n}^3 cell, g = e_x ({tc1 - tc0:.1f} s; scipy.fft workers={threads})")

    out = {
        "metric": "voxel-iters/s & time-to-1e-6 residual: plain vs batched+FNO warm start",
        "value": total_vi / wall,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"stokes3d-{n}^3-overlapping-spheres-r{8 * n // 128}-porosity0.40-seed1"
                               f"-gx/gy/gz-eps{args.eps:g}-plain-single-cell",
                   "cells": 1, "directions": 3, "eps": args.eps, "porosity": round(porosity, 5)},
        "iterations": its,
        "time_to_tol_s": [round(x, 4) for x in secs],
        "K": [[float(v) for v in row] for row in K],
        "iter_us_profiled": round(iter_us_profiled, 2),
        "kernels": per_kernel,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
