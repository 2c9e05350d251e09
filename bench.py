"""Benchmark: batched MLMC Picard-multigrid sample solves per second on one MI355X.

Workload (one "step" = one full pass of the hot path over one batch):
  five MLMC levels on 16^2, 32^2, 64^2, 128^2, 256^2 grids with 4096/1024/256/64/16
  samples (each level >= 1 sample is a fine/coarse pair sharing its KL draw), i.e.
  6816 solves over 6.29 M cells; Gardner infiltration problem, 10 backward-Euler
  steps of dt = 0.01, modified Picard to ||dp||_inf < 1e-8 with one V(2,2) per
  Picard step; KL sampling (64 modes) + all solves + level sums, in one call of
  mlmc_level_estimate.  Inputs are resident on the GPU before timing starts.

Prints one JSON line (see the "value", "roofline" and "cpu_baseline" keys).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Picard-MG sample solves/sec at 1e-8 residual; smoother HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_levels(torch, rmg, W, precision, dev, max_picard):
    from paper_1903_08741_amd import kl_setup
    cfg = W.MLMC_5LEVEL
    f = W.KS_FIELD
    grids = cfg["grids"]
    t0 = time.time()
    _, tables = kl_setup.kl_tables(f["sigma2"], f["corr_len"], f["n_modes"], list(grids))
    log(f"kl basis set-up {time.time() - t0:.1f}s")
    g = W.GARDNER_INFILTRATION
    prob = rmg.Problem(model=rmg.GARDNER, n_steps=g["n_steps"], theta_r=g["theta_r"], theta_s=g["theta_s"],
                       gardner_a=g["gardner_a"], h_top=g["h_top"], h_bottom=g["h_bottom"],
                       h_init=g["h_init"], dt=g["dt"])
    levels = []
    for l, (n, S) in enumerate(zip(grids, cfg["samples"])):
        xi = torch.from_numpy(W.xi_draws(cfg["workload_id"], l, range(S), 1, f["n_modes"])).to(dev)
        levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, fine=prob, coarse=prob,
                           basis_fine=torch.from_numpy(tables[n]).to(dev),
                           basis_coarse=torch.from_numpy(tables[n // 2]).to(dev) if l else None, xi=xi))
    opts = rmg.SolverOpts(precision=precision, max_picard=max_picard)
    marg = [(0.0, f["log_mean"], f["scale"])]
    return levels, opts, marg


def n_solves(levels):
    return sum(lv["xi"].shape[0] * (2 if lv["n_coarse"] else 1) for lv in levels)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    ap.add_argument("--max-picard", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sample-parallel "
              "multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1903_08741_amd as rmg
    import workloads as W

    dev = torch.device("cuda:0")
    precision = rmg.MIXED if args.precision == "mixed" else rmg.FP64
    levels, opts, marg = build_levels(torch, rmg, W, precision, dev, args.max_picard)
    ctx = rmg.default_context(0)
    total = n_solves(levels)
    sums = None
    for i in range(args.warmup):
        t0 = time.time()
        sums, _, rc = ctx.mlmc_level_estimate(levels, marg, opts)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.time() - t0:.3f}s rc={rc}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sums, _, rc = ctx.mlmc_level_estimate(levels, marg, opts)
        log(f"step {i} done rc={rc}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1000.0 * dt / args.steps
    failed = sum(s["n_failed"] for s in sums)
    picard = sum(s["picard_its"] for s in sums)
    out = {
        "metric": METRIC,
        "value": total / (ms / 1000.0),
        "unit": "sample solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 multigrid in f64 Picard" if precision == rmg.MIXED else "f64",
        "data": "synthetic (seeded KL lognormal Ks fields)",
        "config": {"workload": "mlmc 5 levels 16^2..256^2, 4096/1024/256/64/16 samples, Gardner, "
                               "10 steps dt=0.01, V(2,2) per Picard, eps 1e-8",
                   "solves_per_step": total, "cells_per_step": 6291456, "failed_pairs": failed,
                   "picard_iterations_per_step": picard, "precision": args.precision},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
