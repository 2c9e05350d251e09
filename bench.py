"""Benchmark: batched MLMC Picard-multigrid sample solves per second on one MI355X.

Workload (one "step" = one full pass of the hot path over one batch):
  five MLMC levels on 16^2, 32^2, 64^2, 128^2, 256^2 grids with 4096/1024/256/64/16
  samples (each level >= 1 sample is a fine/coarse pair sharing its KL draw), i.e.
  6816 solves over 6.29 M cells; Gardner infiltration problem, 10 backward-Euler
  steps of dt = 0.01, modified Picard to ||dp||_inf < 1e-8 with one V(2,2) per
  Picard step; KL sampling (64 modes) + all solves + level sums, in one call of
  mlmc_level_estimate.  Inputs are resident on the GPU before timing starts.
  Two steps are kept in flight by default (--in-flight): two library contexts, each
  driven by a host thread of its own, share the timed steps, so that one step's
  latency-bound tail (the slowest 256^2 sample's fallback chain, on a few compute
  units) overlaps the other step's work; those calls run unconfined (flag bit 8).
  Every step still does the whole workload and returns the same results; the line
  also reports the rate of the same steps run one after another.

Prints one JSON line (see the "value", "roofline" and "cpu_baseline" keys).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Picard-MG sample solves/sec at 1e-8 residual; smoother HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# LDS peak: 256 compute units x 128 bytes per clock x 2.4 GHz.
LDS_PEAK_BPS = 256 * 128 * 2.4e9
# Access-pattern model of the coarse cycle (FP32, 64^2 -> 4^2, V(2,2)): per cell and level
# visit, nu1 + nu2 = 4 red-black sweeps (the 64^2 and 32^2 levels keep coefficients, right-hand
# side and diagonal in registers: four neighbour reads and one write per update; the coarser
# levels read the five coefficients and the right-hand side from LDS as well: 11 accesses),
# the residual restriction (11 reads per fine cell, a quarter of a coarse cell written twice)
# and the prolongation (one coarse read per fine cell): 32.5 elements per visit on the cached
# levels, 56.5 on the others; the cached levels hold 94 % of the visited cells.
LDS_BYTES_PER_CELL_VISIT = 4 * (0.94 * 32.5 + 0.06 * 56.5)
# Workgroup barriers per coarse cycle on 64^2 -> 4^2 with V(2,2): per level above the coarsest,
# 2 nu1 pre-smoothing half-sweeps, the restriction and 2 nu2 post-smoothing half-sweeps (the
# prolongation is fused into the first); one after the coarsest solve and one after the load.
COARSE_BARRIER_PHASES = 4 * (2 * 2 + 1 + 2 * 2) + 1 + 1
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_down_mlmc5_mixed.md")
KERNEL_SOURCES = ["rmg_smoother.hpp", "rmg_device.hpp", "rmg_internal.hpp"]


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1903_08741_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_record(tag):
    """The last `tag:` line of the committed k_down profile as a dict, or None when there is
    none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            lines = [ln for ln in fh if ln.startswith(tag + ":")]
    except OSError:
        return None
    if not lines:
        return None
    rec = dict(kv.split("=", 1) for kv in lines[-1].split()[1:])
    if rec.get("source_digest") != kernel_source_digest():
        return None
    return rec


def recorded_traffic():
    """HBM bytes per k_down launch from the committed PMC profile (FETCH_SIZE and WRITE_SIZE,
    each scaled by a plain copy's reading), or None when the kernel sources changed since."""
    rec = _profile_record("traffic-record")
    if rec is None:
        return None
    return float(rec["fetch_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])


def recorded_trace_us():
    """Average k_down kernel duration over every launch of the committed kernel trace, or None."""
    rec = _profile_record("trace-record")
    return None if rec is None else float(rec["avg_launch_us"])


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


def build_vg_levels(torch, rmg, W, precision, dev, max_picard):
    """The van Genuchten workload: 5 levels 32^2..512^2 with 2048/512/128/32/8 pairs, three
    KL fields (128 modes each), the infiltration problem of eq. travellingwave with Ks_bl = 0.2,
    50 steps of dt = 0.005, n shifted by (L - l) * 0.1 on level l (the coarse member of a pair
    uses level l - 1's shift)."""
    from paper_1903_08741_amd import kl_setup
    cfg, vf, g = W.MLMC_VG, W.VG_FIELDS, W.VG_INFILTRATION
    grids = cfg["grids"]
    L = len(grids) - 1
    t0 = time.time()
    _, tables = kl_setup.kl_tables(1.0, vf["corr_len"], vf["n_modes"], list(grids) + [grids[0] // 2])
    log(f"kl basis set-up {time.time() - t0:.1f}s")

    def prob(shift):
        return rmg.Problem(model=rmg.VGM, n_steps=g["n_steps"], theta_r=g["theta_r"], theta_s=g["theta_s"],
                           h_top=g["h_top"], h_bottom=g["h_bottom"], h_init=g["h_init"], dt=g["dt"],
                           init_profile=1, init_rate=g["init_rate"], vg_n_shift=shift)
    levels = []
    for l, (n, S) in enumerate(zip(grids, cfg["samples"])):
        xi = torch.from_numpy(W.xi_draws(cfg["workload_id"], l, range(S), 3, vf["n_modes"])).to(dev)
        levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, fine=prob((L - l) * cfg["n_shift_grad"]),
                           coarse=prob((L - l + 1) * cfg["n_shift_grad"]),
                           basis_fine=torch.from_numpy(tables[n]).to(dev),
                           basis_coarse=torch.from_numpy(tables[n // 2]).to(dev) if l else None, xi=xi))
    opts = rmg.SolverOpts(precision=precision, max_picard=max_picard)
    return levels, opts, list(vf["marginals"])


def n_solves(levels):
    return sum(lv["xi"].shape[0] * (2 if lv["n_coarse"] else 1) for lv in levels)


# ------------------------------------------------------- supplementary figures
def grid_classes(levels):
    """Per grid size: the xi rows and basis of every solve on it (fine members of level l,
    coarse members of level l + 1), as the batched call groups them."""
    out = {}
    for l, lv in enumerate(levels):
        out.setdefault(lv["n_fine"], {"basis": lv["basis_fine"], "xi": []})["xi"].append(lv["xi"])
        if lv["n_coarse"]:
            out.setdefault(lv["n_coarse"], {"basis": lv["basis_coarse"], "xi": []})["xi"].append(lv["xi"])
    return out


def per_grid(torch, rmg, ctx, levels, opts, marg, only=None):
    """Each grid's solves alone (one picard_mg_solve call per grid, after one untimed call);
    only: that grid size alone."""
    res = {}
    prob = levels[0]["fine"]
    for n, c in sorted(grid_classes(levels).items()):
        if only is not None and n != only:
            continue
        xi = torch.cat(c["xi"]).contiguous()
        fields = ctx.sample_fields(n, c["basis"], xi, marg)
        ctx.picard_mg_solve(n, fields, prob, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.picard_mg_solve(n, fields, prob, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = out["stats"]["picard_its"]
        ok = int((out["status"] == 0).sum().item())
        res[str(n)] = {"solves": int(xi.shape[0]), "converged": ok, "ms": 1e3 * dt,
                       "solves_per_s": xi.shape[0] / dt, "max_picard_its": int(its.max()),
                       "cell_iterations_per_s": float(its.sum()) * n * n / dt}
        log(f"grid {n}: {1e3 * dt:.1f} ms, max Picard its {int(its.max())}")
    return res


def fp64_path(torch, rmg, ctx, levels, marg, opts, steps=2):
    """The same workload with the multigrid in FP64 too (1 untimed call, `steps` timed)."""
    o = rmg.SolverOpts(**{**opts.__dict__, "precision": rmg.FP64})
    ms, sums = timed_calls(torch, ctx, levels, marg, o, steps)
    failed = sum(s["n_failed"] for s in sums)
    log(f"fp64 path: {ms:.1f} ms per step, failed pairs {failed}")
    return ms, failed


def large_batch_roofline(torch, rmg, ctx, W, levels, marg):
    """The down-leg smoother on a batch large enough to stream from HBM: 64 samples of a
    512 x 512 grid (16.8 M cells, FP32 multigrid arrays ~0.5 GB), 64 Picard iterations of
    one step.  Fields: the 256^2 KL fields of the first 64 draws of the roofline workload,
    each cell repeated on a 2 x 2 block.  The Picard tolerance is set below anything the
    iteration reaches, so that no sample stops early and every launch covers all 64 samples."""
    from paper_1903_08741_amd import _abi
    cfg = W.SMOOTHER_ROOF
    n, S = cfg["n"], cfg["n_samples"]
    c = grid_classes(levels)[n // 2]
    xi = torch.from_numpy(W.xi_draws(cfg["workload_id"], 0, range(S), 1, W.KS_FIELD["n_modes"])).to(c["basis"].device)
    f2 = ctx.sample_fields(n // 2, c["basis"], xi, marg).view(S, 1, n // 2, n // 2)
    fields = f2.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3).reshape(S, 1, n * n).contiguous()
    prob = rmg.Problem(n_steps=1)
    opts = rmg.SolverOpts(precision=rmg.MIXED, max_picard=64, eps_picard=1e-300)
    ctx.picard_mg_solve(n, fields, prob, opts)
    ctx.set_kernel_timing(_abi.TIME_SMOOTHER_DOWN)
    torch.cuda.synchronize()
    ctx.picard_mg_solve(n, fields, prob, opts)
    kt = ctx.kernel_timing()
    ctx.set_kernel_timing(_abi.TIME_NONE)
    gbs = kt["algo_bytes"] / (kt["total_ms"] * 1e-3) / 1e9 if kt["total_ms"] > 0 else 0.0
    log(f"large-batch smoother: {gbs:.0f} GB/s over {kt['launches']} timed launches")
    return {"workload": f"{S} samples of {n}^2, 64 Picard iterations, mixed precision", "bound": "hbm",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "launches": kt["launches"], "avg_launch_us": 1e3 * kt["total_ms"] / max(1, kt["launches"]),
            "algo_bytes_per_launch": kt["algo_bytes"] / max(1, kt["launches"])}


# ----------------------------------------------------------------- CPU baseline
def _oracle_job(args):
    """One oracle solve (twin mode: the same Picard / V-cycle iteration and fallback rule) of a
    workload sample."""
    n, level, i, sopts, Bn = args
    import workloads as W
    from oracle import kl as okl, picard as opicard
    f = W.KS_FIELD
    xi = W.xi_draws(W.MLMC_5LEVEL["workload_id"], level, [i], 1, f["n_modes"])[0, 0]
    Ks = okl.lognormal(okl.gaussian_field(xi, Bn), f["log_mean"], f["scale"]).reshape(n, n)
    t0 = time.perf_counter()
    r = opicard.solve(dict(W.GARDNER_INFILTRATION), {"Ks": Ks}, n, dict(W.SOLVER, **sopts), mode="mg")
    return n, time.perf_counter() - t0, sum(r["picard"]), r["status"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sopts, converged=None, deadline_s=75.0):
    """Time the CPU oracle on a bounded sample of the workload, one solve per worker process.

    Sample: the first draws of the fine member of each level: 32 solves on 16^2, 32 on 32^2,
    16 on 64^2, 8 on 128^2 and 4 on 256^2 (failing and retried draws included, with the
    benchmark's solver settings and fallback rule).  Every grid's mean time per solve is
    measured; the workload's oracle time is (solves per grid) x (mean time per solve), over
    the worker count.  Solves still running at the deadline count with their elapsed time
    (a lower bound on their time), which makes the reported CPU rate an upper bound.
    Converged solves are counted on both sides: the workload's time covers all its solves
    (a failing one costs its iterations too) and the rate counts the solves of converged
    pairs, `converged` (the GPU run's count: the twin oracle takes the same decisions).
    """
    import multiprocessing as mp
    import workloads as W
    from oracle import kl as okl
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    f = W.KS_FIELD
    grids, samples = W.MLMC_5LEVEL["grids"], W.MLMC_5LEVEL["samples"]
    run = {16: 32, 32: 32, 64: 16, 128: 8, 256: 4}
    _, B = okl.basis(f["sigma2"], f["corr_len"], f["n_modes"], list(run), ref_n=64)
    jobs = [(n, grids.index(n), i, sopts, B[n]) for n in sorted(run, reverse=True) for i in range(run[n])]
    env_threads = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    t0 = time.perf_counter()
    pool = mp.get_context("spawn").Pool(min(cores, len(jobs)))
    pending = {k: (jobs[k][0], pool.apply_async(_oracle_job, (jobs[k],))) for k in range(len(jobs))}
    per, unfinished = {}, {}
    while pending and time.perf_counter() - t0 < deadline_s:
        for k in list(pending):
            n, ar = pending[k]
            if ar.ready():
                n_, t, its, st = ar.get()
                per.setdefault(n_, []).append(t)
                del pending[k]
        time.sleep(0.2)
    wall = time.perf_counter() - t0
    for k, (n, _) in pending.items():
        unfinished[n] = unfinished.get(n, 0) + 1
        per.setdefault(n, []).append(wall)  # lower bound of its time
    pool.terminate()
    pool.join()
    if env_threads is None:
        os.environ.pop("OMP_NUM_THREADS", None)
    else:
        os.environ["OMP_NUM_THREADS"] = env_threads
    # solves per grid: the fine members of level l and the coarse members of level l + 1
    counts = {n: samples[l] + (samples[l + 1] if l + 1 < len(grids) else 0) for l, n in enumerate(grids)}
    est = sum(c * sum(per[n]) / len(per[n]) for n, c in counts.items())
    est_wall = est / cores
    total = sum(counts.values())
    counted = total if converged is None else converged
    desc = ", ".join(f"{run[n]}x{n}^2" for n in sorted(run))
    note = ""
    if unfinished:
        note = ("; still running at the " + f"{deadline_s:.0f} s deadline: " +
                ", ".join(f"{k} on {n}^2" for n, k in sorted(unfinished.items())) +
                " (counted at their elapsed time, so the rate is an upper bound)")
    return {"value": counted / est_wall, "unit": "sample solves/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "workers_cap": 16,
            "per_grid_s_per_solve": {str(n): sum(v) / len(v) for n, v in sorted(per.items())},
            "sample": f"{len(jobs)} oracle solves ({desc}; the first draws of each level's fine member, "
                      f"twin mode with the benchmark's solver and fallback settings) in {wall:.1f}s wall on "
                      f"{min(cores, len(jobs))} processes (one per core, at most 16); the {total}-solve "
                      f"workload's time is the per-grid mean time per solve times the solves per grid, "
                      f"divided by the worker count; the rate counts its {counted} solves of converged "
                      f"pairs{note}"}


# ------------------------------------------------------------ adjoint workload
def _oracle_adjoint_job(args):
    """Oracle forward + adjoint (twin multigrid forward, sparse-LU adjoint) of the first
    `steps` steps of one adjoint-workload sample."""
    i, steps, Bn, max_picard = args
    import workloads as W
    from oracle import adjoint as oadj, kl as okl
    cfg, f = W.ADJOINT_128, W.KS_FIELD
    n = cfg["n"]
    xi = W.xi_draws(cfg["workload_id"], 0, [i], 1, cfg["n_modes"])[0, 0]
    Ks = okl.lognormal(okl.gaussian_field(xi, Bn), f["log_mean"], f["scale"]).reshape(n, n)
    t0 = time.perf_counter()
    r = oadj.solve_with_gradient(dict(W.GARDNER_INFILTRATION, n_steps=steps), Ks, n,
                                 dict(W.SOLVER, max_picard=max_picard), basis=Bn, mode="mg")
    return time.perf_counter() - t0, r["status"]


def adjoint_cpu_baseline(max_picard, steps=2):
    """The oracle adjoint on a bounded sample: the first `steps` of the 20 steps of 16
    samples, one process per core; the full workload's time is that per-sample time
    scaled by 20 / steps, times the sample count, over the worker count."""
    import multiprocessing as mp
    import workloads as W
    from oracle import kl as okl
    cfg, f = W.ADJOINT_128, W.KS_FIELD
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    _, B = okl.basis(f["sigma2"], f["corr_len"], cfg["n_modes"], [cfg["n"]], ref_n=64)
    jobs = [(i, steps, B[cfg["n"]], max_picard) for i in range(16)]
    env_threads = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(min(cores, len(jobs))) as pool:
        res = list(pool.imap_unordered(_oracle_adjoint_job, jobs, chunksize=1))
    wall = time.perf_counter() - t0
    if env_threads is None:
        os.environ.pop("OMP_NUM_THREADS", None)
    else:
        os.environ["OMP_NUM_THREADS"] = env_threads
    per_sample = sum(t for t, _ in res) / len(res) * (cfg["n_steps"] / steps)
    est_wall = per_sample * cfg["n_samples"] / cores
    return {"value": cfg["n_samples"] / est_wall, "unit": "sample gradients/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle forward (twin multigrid) + adjoint (sparse LU) of the first {steps} of "
                      f"{cfg['n_steps']} steps of 16 samples in {wall:.1f}s wall on {min(cores, len(jobs))} "
                      f"processes; scaled by {cfg['n_steps']}/{steps} steps and {cfg['n_samples']} samples "
                      "over the worker count"}


def adjoint_bench(args, torch, rmg, W):
    """The adjoint workload: 1024 samples of 128^2, 100 KL modes, 20 steps, checkpoints every
    5 steps; one step = one picard_mg_adjoint call (fields, forward with checkpoints,
    segment recomputation, adjoint sweep, dQ/dxi)."""
    from paper_1903_08741_amd import _abi, kl_setup
    cfg, f, g = W.ADJOINT_128, W.KS_FIELD, W.GARDNER_INFILTRATION
    dev = torch.device("cuda:0")
    n, S, M = cfg["n"], cfg["n_samples"], cfg["n_modes"]
    _, tables = kl_setup.kl_tables(f["sigma2"], f["corr_len"], M, [n])
    B = torch.from_numpy(tables[n]).to(dev)
    xi = torch.from_numpy(W.xi_draws(cfg["workload_id"], 0, range(S), 1, M)[:, 0, :].copy()).to(dev)
    prob = rmg.Problem(model=rmg.GARDNER, n_steps=cfg["n_steps"], theta_r=g["theta_r"], theta_s=g["theta_s"],
                       gardner_a=g["gardner_a"], h_top=g["h_top"], h_bottom=g["h_bottom"], h_init=g["h_init"],
                       dt=g["dt"])
    marg = (0.0, f["log_mean"], f["scale"])
    # absolute tolerance on the multipliers' corrections: they are ~1e-4 in this workload
    # (dt times the outflux sensitivity), so 1e-13 converges them to ~1e-9 relative
    eps_adj = 1e-13
    precision = rmg.MIXED if args.precision == "mixed" else rmg.FP64
    opts = rmg.SolverOpts(precision=precision, max_picard=args.max_picard, fallback_cycles=args.fallback_cycles,
                          fallback_max_picard=args.fallback_max_picard if args.fallback_cycles else 0)
    if args.no_autotune:
        opts.flags |= rmg.FLAG_NO_AUTOTUNE
    ctx = rmg.default_context(0)

    def call(o):
        return ctx.picard_mg_adjoint(n, B, xi, marg, prob, o, ckpt_every=cfg["ckpt_every"], eps_adjoint=eps_adj)
    for i in range(args.warmup):
        t0 = time.time()
        out = call(opts)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.time() - t0:.3f}s rc={out['rc']}")
    ctx.set_kernel_timing(_abi.TIME_SMOOTHER_DOWN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = call(opts)
        log(f"step {i} done rc={out['rc']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1000.0 * dt / args.steps
    kt = ctx.kernel_timing()
    ctx.set_kernel_timing(_abi.TIME_NONE)
    ok = out["status"] == 0
    n_ok = int(ok.sum().item())
    fwd, adj = out["stats_forward"], out["stats_adjoint"]
    gbs = kt["algo_bytes"] / (kt["total_ms"] * 1e-3) / 1e9 if kt["total_ms"] > 0 else 0.0
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_down (nu1 fused red-black sweeps + residual + restriction), forward and adjoint sweeps",
            "launches": kt["launches"], "avg_launch_us": 1e3 * kt["total_ms"] / max(1, kt["launches"]),
            "algo_bytes_per_launch": kt["algo_bytes"] / max(1, kt["launches"])}
    extras = {}
    if not args.no_extras and precision == rmg.MIXED:
        o64 = rmg.SolverOpts(**{**opts.__dict__, "precision": rmg.FP64})
        call(o64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ref = call(o64)
        torch.cuda.synchronize()
        ms64 = 1e3 * (time.perf_counter() - t1)
        both = ok & (ref["status"] == 0)
        gm, gr = out["grad"][both], ref["grad"][both]
        rel = ((gm - gr).abs().amax(dim=1) / gr.abs().amax(dim=1)).cpu()
        qrel = ((out["q"][both] - ref["q"][both]).abs() / ref["q"][both].abs()).cpu()
        extras["fp64_path"] = {"ms_per_step": ms64, "mixed_speedup": ms64 / ms,
                               "samples_compared": int(both.sum().item()),
                               "grad_rel_err_max": float(rel.max()) if rel.numel() else None,
                               "grad_rel_err_median": float(rel.median()) if rel.numel() else None,
                               "q_rel_err_max": float(qrel.max()) if qrel.numel() else None}
        log(f"fp64 adjoint: {ms64:.1f} ms; grad rel err max {extras['fp64_path']['grad_rel_err_max']}")
    cpu = None
    if not args.no_cpu_baseline:
        t1 = time.time()
        cpu = adjoint_cpu_baseline(args.max_picard)
        log(f"cpu baseline {time.time() - t1:.1f}s")
    res = {
        "metric": "Picard-MG adjoint sample gradients/sec (dQ/dxi, 100 KL coefficients)",
        "value": n_ok / (ms / 1000.0),
        "unit": "sample gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 multigrid in f64 Picard and f64 adjoint residual" if precision == rmg.MIXED else "f64",
        "data": "synthetic (seeded KL lognormal Ks fields)",
        "config": {"workload": f"adjoint: {S} samples of {n}^2, Gardner, {M} KL modes, {cfg['n_steps']} steps "
                               f"dt=0.01, QoI time-integrated bottom outflux, checkpoints every "
                               f"{cfg['ckpt_every']} steps, V(2,2) per Picard / adjoint iteration, "
                               f"eps 1e-8 forward, {eps_adj:g} adjoint",
                   "samples": S, "converged_samples": n_ok,
                   "forward_picard_iterations": int(fwd["picard_its"].sum()),
                   "adjoint_iterations": int(adj["picard_its"].sum()),
                   "precision": args.precision, "max_picard": args.max_picard},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    res.update(extras)
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------ adaptive PC_MLMC
def pcmlmc_bench(args, torch, rmg, W):
    """Algorithm 1 (pc_mlmc) with parametric continuation, cost in work units.  One step = one
    whole adaptive run (warm-up, updates of N_l, all batches).

    gardner (default): the Gardner problem of the MLMC workload on levels 16^2 .. 16 * 2^(L-1)
    with the exponent a as the continuation parameter, a_l = 1 - 0.1 (L - 1 - l);
    vg: the van Genuchten fields of the vg workload (infiltration problem of eq. travellingwave,
    Ks_bl = 0.2) on levels 32^2 .. 32 * 2^(L-1) with n shifted by (L - 1 - l) * 0.1, 100 steps to
    T = 0.25 (dt = 0.0025); the sampling tolerance is RMSE / sqrt(2), so that an eq. discErr bias
    estimate below RMSE / sqrt(2) as well meets the RMSE target (eq. errMLMC)."""
    from paper_1903_08741_amd import _abi, kl_setup
    dev = torch.device("cuda:0")
    L = args.levels
    vg = args.pc_model == "vg"
    if vg:
        cfg, vf, g = W.PC_MLMC_VG, W.VG_FIELDS, W.VG_INFILTRATION
        grids = cfg["grids"][:L]
        _, tables = kl_setup.kl_tables(1.0, vf["corr_len"], vf["n_modes"], list(grids) + [grids[0] // 2])
        F, M, marg, wid = 3, vf["n_modes"], list(vf["marginals"]), cfg["workload_id"]
        warm = cfg["warmup"]
        steps = args.time_steps or cfg["n_steps_full"]
        dt = g["n_steps"] * g["dt"] / steps
        eps = args.eps or args.rmse / 2 ** 0.5

        def prob(l):
            return rmg.Problem(model=rmg.VGM, n_steps=steps, theta_r=g["theta_r"], theta_s=g["theta_s"],
                               h_top=g["h_top"], h_bottom=g["h_bottom"], h_init=g["h_init"], dt=dt,
                               init_profile=1, init_rate=g["init_rate"],
                               vg_n_shift=(L - 1 - l) * cfg["n_shift_grad"])
        theta = (f"infiltration problem, n shifted by (L-1-l)*{cfg['n_shift_grad']}, {steps} steps dt={dt:g}, "
                 f"RMSE target {args.rmse:g}")
    else:
        f, g = W.KS_FIELD, W.GARDNER_INFILTRATION
        grids = tuple(16 << l for l in range(L))
        _, tables = kl_setup.kl_tables(f["sigma2"], f["corr_len"], f["n_modes"], list(grids) + [8])
        F, M, marg, wid = 1, f["n_modes"], [(0.0, f["log_mean"], f["scale"])], 6
        warm = (64, 32, 16, 8, 8, 4)
        eps = args.eps or 2e-3

        def prob(l):
            return rmg.Problem(model=rmg.GARDNER, n_steps=g["n_steps"], theta_r=g["theta_r"], theta_s=g["theta_s"],
                               gardner_a=1.0 - 0.1 * (L - 1 - l), h_top=g["h_top"], h_bottom=g["h_bottom"],
                               h_init=g["h_init"], dt=g["dt"])
        theta = f"Gardner a_l = 1 - 0.1 (L-1-l), {g['n_steps']} steps dt={g['dt']}"
    levels = []
    for l, n in enumerate(grids):
        levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, n_warmup=warm[l], fine=prob(l),
                           coarse=prob(l - 1) if l else None,
                           basis_fine=torch.from_numpy(tables[n]).to(dev),
                           basis_coarse=torch.from_numpy(tables[n // 2]).to(dev) if l else None))

    def src(level, first, count):
        log(f"  draw level {level}: pairs {first}..{first + count - 1}")
        return W.xi_draws(wid, level, range(first, first + count), F, M)
    ctx = rmg.default_context(0)
    precision = rmg.MIXED if args.precision == "mixed" else rmg.FP64

    def run(prec):
        opts = rmg.SolverOpts(precision=prec, max_picard=args.max_picard, fallback_cycles=args.fallback_cycles,
                              fallback_max_picard=args.fallback_max_picard if args.fallback_cycles else 0)
        return ctx.pc_mlmc(levels, marg, opts, eps, src, max_rounds=50, max_pairs=args.max_pairs)
    for i in range(args.warmup):
        run(precision)
        torch.cuda.synchronize()
    ctx.set_kernel_timing(_abi.TIME_SMOOTHER_DOWN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = run(precision)
        log(f"step {i} done rc={r['rc']} rounds={r['rounds']}")
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    kt = ctx.kernel_timing()
    ctx.set_kernel_timing(_abi.TIME_NONE)
    gbs = kt["algo_bytes"] / (kt["total_ms"] * 1e-3) / 1e9 if kt["total_ms"] > 0 else 0.0
    solves = sum(x["drawn"] * (2 if l else 1) for l, x in enumerate(r["levels"]))
    lv = [{"grid": grids[l], "pairs_drawn": x["drawn"], "successful": x["sums"]["n"], "failed": x["sums"]["n_failed"],
           "retried": x["sums"]["n_retried"], "N_l": x["target"], "W_l": x["W"], "V_l": x["V"], "mean_Y": x["mean"]}
          for l, x in enumerate(r["levels"])]
    rmse = (r["bias"] ** 2 + r["sampling_err2"]) ** 0.5 if L > 1 else r["sampling_err2"] ** 0.5
    extras = {}
    if not args.no_extras and precision == rmg.MIXED:
        t1 = time.perf_counter()
        r64 = run(rmg.FP64)
        extras["fp64_path"] = {"ms": 1e3 * (time.perf_counter() - t1), "mean": r64["mean"],
                               "sampling_err": r64["sampling_err2"] ** 0.5,
                               "mean_difference": r["mean"] - r64["mean"],
                               "pairs_drawn": [x["drawn"] for x in r64["levels"]]}
    res = {
        "metric": "PC_MLMC wall time to the sampling tolerance (Algorithm 1)",
        "value": ms / 1000.0, "unit": "s per adaptive run", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 multigrid in f64 Picard" if precision == rmg.MIXED else "f64",
        "data": "synthetic (seeded KL fields)",
        "config": {"workload": f"PC_MLMC, {'van Genuchten-Mualem' if vg else 'Gardner'}, {L} levels "
                               f"{grids[0]}^2..{grids[-1]}^2, {theta}, eps {eps:g}, work cost model, "
                               f"V(2,2) per Picard, eps_PI 1e-8, at most {args.max_pairs} pairs per level",
                   "levels": lv, "rounds": r["rounds"], "calls": r["calls"], "solves": solves,
                   "converged": bool(r["converged"]), "rc": r["rc"], "precision": args.precision,
                   "max_picard": args.max_picard},
        "estimate": {"mean": r["mean"], "var": r["var"], "sampling_err": r["sampling_err2"] ** 0.5,
                     "bias_estimate": r["bias"], "rmse_estimate": rmse},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "k_down over every batch of the run",
                     "launches": kt["launches"], "avg_launch_us": 1e3 * kt["total_ms"] / max(1, kt["launches"])},
        "cpu_baseline": None,
    }
    res.update(extras)
    print(json.dumps(res), flush=True)


def pcmlmc_eps_sweep(args, torch, rmg, W):
    """Cost of Algorithm 1 against the tolerance (Section 6: with h_L proportional to eps the
    estimator's cost grows like the cost of one deterministic solve on the finest grid).  The
    Gardner hierarchy of pcmlmc_bench; the tolerance is halved while the finest grid is refined
    by one level: (eps, L) = (1.6e-2, 2), (8e-3, 3), (4e-3, 4), (2e-3, 5), levels 16^2 .. 16 * 2^(L-1).
    Cost is reported in work units (the sum over levels of pairs x Picard-MG cycles x cells) and in
    wall time; the exponent is the least-squares slope of log(cost) against log(1 / eps).  With a
    fixed number of time steps the work of one finest solve grows like h_L^-2 times its iteration
    count (the paper refines the time step with the mesh as well, hence its eps^-3)."""
    from paper_1903_08741_amd import kl_setup
    dev = torch.device("cuda:0")
    f, g = W.KS_FIELD, W.GARDNER_INFILTRATION
    points = [(1.6e-2, 2), (8e-3, 3), (4e-3, 4), (2e-3, 5)]
    all_grids = tuple(16 << l for l in range(max(L for _, L in points)))
    _, tables = kl_setup.kl_tables(f["sigma2"], f["corr_len"], f["n_modes"], list(all_grids) + [8])
    marg = [(0.0, f["log_mean"], f["scale"])]
    warm = (64, 32, 16, 8, 8, 4)
    ctx = rmg.default_context(0)
    precision = rmg.MIXED if args.precision == "mixed" else rmg.FP64
    out = []
    for eps, L in points:
        def prob(l, L=L):
            return rmg.Problem(model=rmg.GARDNER, n_steps=g["n_steps"], theta_r=g["theta_r"], theta_s=g["theta_s"],
                               gardner_a=1.0 - 0.1 * (L - 1 - l), h_top=g["h_top"], h_bottom=g["h_bottom"],
                               h_init=g["h_init"], dt=g["dt"])
        levels = []
        for l in range(L):
            n = all_grids[l]
            levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, n_warmup=warm[l], fine=prob(l),
                               coarse=prob(l - 1) if l else None,
                               basis_fine=torch.from_numpy(tables[n]).to(dev),
                               basis_coarse=torch.from_numpy(tables[n // 2]).to(dev) if l else None))

        def src(level, first, count, L=L):
            return W.xi_draws(100 + L, level, range(first, first + count), 1, f["n_modes"])
        opts = rmg.SolverOpts(precision=precision, max_picard=args.max_picard,
                              fallback_cycles=args.fallback_cycles,
                              fallback_max_picard=args.fallback_max_picard if args.fallback_cycles else 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.pc_mlmc(levels, marg, opts, eps, src, max_rounds=50, max_pairs=args.max_pairs)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        pt = {"eps": eps, "levels": L, "finest": all_grids[L - 1], "work": r["total_cost"], "wall_ms": ms,
              "N_l": [x["target"] for x in r["levels"]], "pairs_drawn": [x["drawn"] for x in r["levels"]],
              "W_finest": r["levels"][-1]["W"],
              "sampling_err": r["sampling_err2"] ** 0.5, "bias_estimate": r["bias"], "mean": r["mean"],
              "converged": bool(r["converged"]), "rc": r["rc"]}
        log(f"eps {eps:g} L {L}: work {r['total_cost']:.4g}, {ms:.0f} ms, N_l {pt['N_l']}, "
            f"sampling err {pt['sampling_err']:.3g}, bias {r['bias']:.3g}")
        out.append(pt)
    x = np.log([1.0 / p["eps"] for p in out])

    def slope(y):
        y = np.log(y)
        return float(np.polyfit(x, y, 1)[0])
    res = {
        "metric": "PC_MLMC cost against the tolerance (Algorithm 1, h_L ~ eps)",
        "value": slope([p["work"] for p in out]), "unit": "exponent of work in 1/eps", "n_gpus": 1,
        "steps": len(out), "warmup": 0, "ms_per_step": float(np.mean([p["wall_ms"] for p in out])),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32 multigrid in f64 Picard" if precision == rmg.MIXED else "f64",
        "data": "synthetic (seeded KL fields)",
        "config": {"workload": f"PC_MLMC eps sweep, Gardner a_l = 1 - 0.1 (L-1-l), {g['n_steps']} steps "
                               f"dt={g['dt']}, levels 16^2..16*2^(L-1), work cost model",
                   "points": out},
        "wall_time_exponent": slope([p["wall_ms"] for p in out]),
        "finest_solve_work_exponent": slope([p["W_finest"] for p in out]),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------ KL field sampling
def kl_bench(args, torch, rmg, W):
    """The KL field sampling kernel (FP64 matrix-core GEMM G = xi B plus the lognormal
    transform) at the two shapes the workloads sample: the adjoint workload's 1024 samples
    of 128^2 with 100 modes, and the 5-level MLMC call's fields (every grid's fine and coarse
    members, 64 modes).  One step = both shapes once.  FLOPs: 2 rows x modes x cells per
    call (the exp epilogue not counted); bytes: basis + coefficients in, fields out."""
    from paper_1903_08741_amd import kl_setup
    dev = torch.device("cuda:0")
    f = W.KS_FIELD
    marg = [(0.0, f["log_mean"], f["scale"])]
    jobs = []
    cfg = W.ADJOINT_128
    _, t3 = kl_setup.kl_tables(f["sigma2"], f["corr_len"], cfg["n_modes"], [cfg["n"]])
    jobs.append((cfg["n"], torch.from_numpy(t3[cfg["n"]]).to(dev),
                 torch.from_numpy(W.xi_draws(cfg["workload_id"], 0, range(cfg["n_samples"]), 1,
                                             cfg["n_modes"])).to(dev)))
    grids, samples = W.MLMC_5LEVEL["grids"], W.MLMC_5LEVEL["samples"]
    _, t1 = kl_setup.kl_tables(f["sigma2"], f["corr_len"], f["n_modes"], list(grids))
    for l, n in enumerate(grids):
        S = samples[l] + (samples[l + 1] if l + 1 < len(grids) else 0)
        jobs.append((n, torch.from_numpy(t1[n]).to(dev),
                     torch.from_numpy(W.xi_draws(W.MLMC_5LEVEL["workload_id"], l, range(S), 1,
                                                 f["n_modes"])).to(dev)))
    outs = [torch.empty((x.shape[0], 1, n * n), dtype=torch.float64, device=dev) for n, _, x in jobs]
    ctx = rmg.default_context(0)

    def step():
        for (n, B, x), o in zip(jobs, outs):
            ctx.sample_fields(n, B, x, marg, out=o)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(jobs))]
    per = [0.0] * len(jobs)
    for _ in range(args.steps):
        for k, ((n, B, x), o) in enumerate(zip(jobs, outs)):
            ev[2 * k].record()
            ctx.sample_fields(n, B, x, marg, out=o)
            ev[2 * k + 1].record()
        torch.cuda.synchronize()
        for k in range(len(jobs)):
            per[k] += ev[2 * k].elapsed_time(ev[2 * k + 1])
    rows = []
    tot_ms = tot_flop = tot_bytes = 0.0
    for k, (n, B, x) in enumerate(jobs):
        ms = per[k] / args.steps
        S, M, N = x.shape[0], x.shape[2], n * n
        flop = 2.0 * S * M * N
        byt = 8.0 * (M * N + S * M + S * N)
        rows.append({"n": n, "rows": S, "modes": M, "ms": ms, "tflops": flop / ms / 1e9, "gbs": byt / ms / 1e6})
        tot_ms, tot_flop, tot_bytes = tot_ms + ms, tot_flop + flop, tot_bytes + byt
    big = rows[0]
    res = {
        "metric": "KL field sampling FP64 matrix-core TFLOP/s (G = xi B, then exp)",
        "value": big["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": tot_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded standard normals; KL bases of the workloads)",
        "config": {"workload": "sample_fields: 1024 x 100 modes x 128^2 (the adjoint workload) and the 5-level "
                               "MLMC call's fields (64 modes, 16^2..256^2)", "shapes": rows,
                   "mlmc_fields_ms": sum(r["ms"] for r in rows[1:])},
        "roofline": {"bound": "mfma", "achieved": big["tflops"], "peak": 78.6, "unit": "TFLOP/s",
                     "frac": big["tflops"] / 78.6, "traffic": None, "kernel": "k_kl_fields (1024 x 100 x 16384)",
                     "hbm_gbs": big["gbs"]},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------ robustness sweep
def sweep_bench(args, torch, rmg, W):
    """Section 4.3's robustness sweep as one batched solve: the 20 x 20 (alpha, n) pairs of
    Table alpha_n times 64 Ks fields (the same 64 draws for every pair), the infiltration
    problem of eq. travellingwave, W(2,2) cycles to eps_MG = 1e-5, eps_PI = 1e-5, at most 50
    Picard iterations per step.  Reports the cost map (mean W-cycles to T_final over the
    converged samples of a pair) and the failure map (failed samples out of 64)."""
    from paper_1903_08741_amd import kl_setup
    cfg, tw = W.SWEEP, W.TRAVELLING_WAVE
    dev = torch.device("cuda:0")
    P, M = cfg["samples_per_pair"], cfg["n_modes"]
    n = args.sweep_h
    dt = 1.0 / args.sweep_dt
    n_steps = int(np.ceil(W.SWEEP_T_FINAL / dt - 1e-9))  # first multiple of dt at or past T_final
    phi = W.MATERN_PHI1 if args.sweep_phi == 1 else W.MATERN_PHI2
    A, NV = W.SWEEP_ALPHA, W.SWEEP_N
    _, tables = kl_setup.kl_tables(0.0, 0.0, M, [n], matern_phi=phi)
    ctx = rmg.default_context(0)
    B = torch.from_numpy(tables[n]).to(dev)
    xi = torch.from_numpy(W.xi_draws(cfg["workload_id"], 0, range(P), 1, M)).to(dev)
    ks = ctx.sample_fields(n, B, xi, [(0.0, float(np.log(tw["ks_baseline"])), 1.0)])[:, 0]  # [P][N]
    pairs = [(a, v) for a in A for v in NV]
    S = len(pairs) * P
    fields = torch.empty(S, 3, n * n, dtype=torch.float64, device=dev)
    fields[:, 0] = ks.repeat(len(pairs), 1)
    av = torch.tensor([a for a, _ in pairs], dtype=torch.float64, device=dev).repeat_interleave(P)
    nv = torch.tensor([v for _, v in pairs], dtype=torch.float64, device=dev).repeat_interleave(P)
    fields[:, 1] = av[:, None]
    fields[:, 2] = nv[:, None]
    prob = rmg.Problem(model=rmg.VGM, n_steps=n_steps, theta_r=tw["theta_r"], theta_s=tw["theta_s"],
                       h_top=tw["h_top"], h_bottom=tw["h_bottom"], h_init=tw["h_init"], dt=dt,
                       init_profile=1, init_rate=tw["init_rate"])
    precision = rmg.MIXED if args.precision == "mixed" else rmg.FP64
    opts = rmg.SolverOpts(precision=precision, cycle=rmg.CYCLE_W, cycles_per_picard=0, eps_mg=cfg["eps_mg"],
                          eps_picard=cfg["eps"], max_picard=cfg["max_picard"])
    for i in range(args.warmup):
        ctx.picard_mg_solve(n, fields, prob, opts)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = ctx.picard_mg_solve(n, fields, prob, opts)
        log(f"step {i} done rc={out['rc']}")
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    st = out["status"].cpu().numpy().reshape(len(A), len(NV), P)
    cyc = out["stats"]["mg_cycles"].reshape(len(A), len(NV), P).astype(np.float64)
    ok = st == 0
    with np.errstate(invalid="ignore"):
        cost = np.where(ok.any(axis=2), (cyc * ok).sum(axis=2) / np.maximum(ok.sum(axis=2), 1), np.nan)
    fails = (~ok).sum(axis=2)
    res = {
        "metric": "Picard-MG robustness sweep sample solves/sec (W(2,2) to eps_MG, Table alpha_n)",
        "value": float(ok.sum()) / (ms / 1000.0), "unit": "sample solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 multigrid in f64 Picard" if precision == rmg.MIXED else "f64",
        "data": f"synthetic (seeded Matern Phi_{args.sweep_phi} KL Ks fields; alpha, n from Table alpha_n)",
        "config": {"workload": f"robustness sweep: {len(A)}x{len(NV)} (alpha, n) pairs x {P} Ks fields = {S} "
                               f"solves of {n}^2 (h=1/{n}), Matern Phi_{args.sweep_phi}, vG, infiltration "
                               f"problem, {n_steps} steps dt=1/{args.sweep_dt}, W(2,2) to eps_MG 1e-5, "
                               "eps_PI 1e-5, at most 50 Picard iterations",
                   "h": f"1/{n}", "dt": f"1/{args.sweep_dt}", "phi": args.sweep_phi,
                   "solves": S, "converged": int(ok.sum()), "precision": args.precision},
        "roofline": None,
        "cpu_baseline": None,
        "alpha": list(A), "n": list(NV),
        "mean_w_cycles": [[None if np.isnan(x) else round(float(x), 1) for x in row] for row in cost],
        "failures_of_64": fails.tolist(),
    }
    print(json.dumps(res), flush=True)


def tuned_schedule(ctx):
    """The library's tuning choices after the timed calls: streaming tile edges per grid, and
    for the batched call the compute-unit confinement and the passes per graph batch."""
    out = {"tiles": {}, "batched_call": None}
    for sig, val in ctx.tune_choices().items():
        v = [int(x) for x in val.split()]
        if sig.startswith("tiles "):
            n = sig.split()[1].split("=")[1]
            out["tiles"][n] = v
        elif sig.startswith("sched ") and len(v) == 2:
            flags = sig.rsplit("flags=", 1)[-1]
            key = "batched_call" if flags == "0" else f"batched_call_flags_{flags}"
            out[key] = {"confine": bool(v[0]), "passes_per_batch": v[1]}
    return out


def level_report(sums, levels):
    """Per level: pairs, failed and retried pairs with their fractions, and the level mean."""
    out = []
    for l, (sm, lv) in enumerate(zip(sums, levels)):
        S = int(lv["xi"].shape[0])
        hi, lo = sm["sY"]
        out.append({"level": l, "grid": lv["n_fine"], "pairs": S, "failed": sm["n_failed"],
                    "failed_fraction": sm["n_failed"] / S, "retried": sm["n_retried"],
                    "retried_fraction": sm["n_retried"] / S,
                    "mean_Y": (hi + lo) / sm["n"] if sm["n"] else None, "picard_its": sm["picard_its"]})
    return out


def timed_calls(torch, ctx, levels, marg, opts, steps=1):
    """One untimed call, then `steps` timed ones: (ms per call, level sums of the last)."""
    ctx.mlmc_level_estimate(levels, marg, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sums, _, _ = ctx.mlmc_level_estimate(levels, marg, opts)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps, sums


def extra_contexts(rmg, ctx, n, tune_cache):
    """n more contexts on device 0 that start with ctx's tuning choices: the tune-cache file
    when one is given (ctx has written its choices there), else a temporary copy of them."""
    import tempfile
    if tune_cache:
        return [rmg.Context(0, tune_cache=tune_cache) for _ in range(n)]
    fd, path = tempfile.mkstemp(prefix="rmg_tune_", suffix=".txt")
    try:
        with os.fdopen(fd, "w") as fh:
            fh.write(ctx.tune_text())
        return [rmg.Context(0, tune_cache=path) for _ in range(n)]
    finally:
        os.unlink(path)


def torch_side_stream(torch):
    """A context manager that puts the calling thread's torch work on a new stream and waits
    for that stream on exit."""
    import contextlib

    @contextlib.contextmanager
    def on_stream():
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            yield
        st.synchronize()
    return on_stream


def in_flight_counts(steps, P):
    """Steps per context when `steps` are dealt out over P contexts (the first ones take one
    more when P does not divide steps)."""
    return [steps // P + (1 if j < steps % P else 0) for j in range(P)]


def run_in_flight(torch, ctxs, steps, call, on_stream=None):
    """`steps` calls dealt out over the contexts, each context driven by a host thread of its
    own on a stream of its own (on_stream; default a new torch stream per thread).  A context
    is not thread safe; separate contexts share nothing, so their calls overlap on the GPU.
    Returns the results of every call (context by context); an exception in any thread is
    re-raised here after every thread has ended."""
    import threading
    on_stream = on_stream or torch_side_stream(torch)
    P = len(ctxs)
    counts = in_flight_counts(steps, P)
    outs = [[] for _ in range(P)]
    errs = []

    def worker(j):
        try:
            with on_stream():
                for i in range(counts[j]):
                    outs[j].append(call(ctxs[j]))
                    log(f"step done (context {j}, {i + 1} of {counts[j]})")
        except BaseException as e:  # re-raised in the calling thread
            errs.append(e)

    th = [threading.Thread(target=worker, args=(j,)) for j in range(P) if counts[j]]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errs:
        raise errs[0]
    return [r for o in outs for r in o]


def same_results(torch, runs):
    """Whether every call returned the same level sums and bit-identical QoIs."""
    s0, q0 = runs[0][0], runs[0][1]
    return all(s == s0 and torch.equal(q.view(torch.int64), q0.view(torch.int64)) for s, q, _ in runs)


def solver_variants(torch, rmg, ctx, levels, marg, base, total):
    """The same workload under other solver settings (outside the timed region): one V(2,2)
    per Picard step without the fallback (failed pairs dropped), two V(2,2) per step, one
    W(2,2) per step.  Converged solves per second and failures per level."""
    out = []
    for name, kw in (("V(2,2) x1, no fallback, limit 500", dict(cycles_per_picard=1, max_picard=500,
                                                                 fallback_cycles=0, fallback_max_picard=0)),
                     ("V(2,2) x2, no fallback, limit 500", dict(cycles_per_picard=2, max_picard=500,
                                                                 fallback_cycles=0, fallback_max_picard=0)),
                     ("W(2,2) x1, no fallback, limit 500", dict(cycle=rmg.CYCLE_W, cycles_per_picard=1,
                                                                 max_picard=500, fallback_cycles=0,
                                                                 fallback_max_picard=0))):
        o = rmg.SolverOpts(**{**base.__dict__, **kw})
        ms, sums = timed_calls(torch, ctx, levels, marg, o)
        conv = sum(sm["n"] * (2 if lv["n_coarse"] else 1) for sm, lv in zip(sums, levels))
        out.append({"solver": name, "ms_per_step": ms, "converged_solves": conv, "solves": total,
                    "converged_solves_per_s": conv / (ms / 1e3),
                    "failed_pairs_per_level": [sm["n_failed"] for sm in sums]})
        log(f"variant {name}: {ms:.1f} ms, failed {[sm['n_failed'] for sm in sums]}")
    return out


def coarse_bound(kt, levels_visited_per_launch=None):
    """Bound line of the one-workgroup-per-sample coarse cycle: level cells per second,
    the LDS traffic of its access pattern against the LDS peak, and the time per barrier
    phase (the kernel is a chain of short barrier-separated phases per sample)."""
    if kt["total_ms"] <= 0 or kt["launches"] == 0:
        return None
    sec = kt["total_ms"] * 1e-3
    cells_s = kt["cells"] / sec
    lds_b = LDS_BYTES_PER_CELL_VISIT * kt["cells"]
    return {"bound": "latency (LDS + barriers)", "kernel": "k_coarse_v (64^2 -> 4^2 cycle in LDS, one workgroup "
                                                          "per sample)",
            "launches": kt["launches"], "avg_launch_us": 1e3 * kt["total_ms"] / kt["launches"],
            "level_cells_per_s": cells_s, "lds_bytes_per_s_model": lds_b / sec,
            "lds_peak_bytes_per_s": LDS_PEAK_BPS, "lds_frac": lds_b / sec / LDS_PEAK_BPS,
            "lds_bytes_per_cell_visit_model": LDS_BYTES_PER_CELL_VISIT,
            "barrier_phases_per_cycle": COARSE_BARRIER_PHASES}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("gardner", "vg", "adjoint", "sweep", "pcmlmc", "kl"), default="gardner",
                    help="gardner: the 5-level Gardner MLMC workload (default); vg: the van Genuchten "
                         "workload with three fields and continuation (5 levels 32^2..512^2, infiltration "
                         "problem); adjoint: outflux gradients of 1024 samples of 128^2 (100 KL modes, 20 "
                         "steps); sweep: the alpha-n robustness sweep of the infiltration problem (25600 "
                         "solves of 32^2); pcmlmc: Algorithm 1")
    ap.add_argument("--levels", type=int, default=4, help="pcmlmc: number of levels (at most 6)")
    ap.add_argument("--eps", type=float, default=0.0,
                    help="pcmlmc: sampling tolerance (default: 2e-3 for gardner; RMSE / sqrt(2) for vg)")
    ap.add_argument("--rmse", type=float, default=1e-3, help="pcmlmc vg: target RMSE")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="pcmlmc vg: backward-Euler steps to T = 0.25 (default 100)")
    ap.add_argument("--pc-model", choices=("gardner", "vg"), default="gardner", help="pcmlmc: hierarchy")
    ap.add_argument("--max-pairs", type=int, default=50000, help="pcmlmc: cap on the pairs drawn per level")
    ap.add_argument("--grid", type=int, default=0,
                    help="gardner: solve only this grid size's class of the MLMC workload (one untimed and "
                         "one timed call; for profiling one class)")
    ap.add_argument("--sweep-h", type=int, choices=(32, 64), default=32,
                    help="sweep: cells per side (h = 1/32 or 1/64, the two grids of Section 4.3)")
    ap.add_argument("--sweep-dt", type=int, choices=(64, 128), default=64,
                    help="sweep: time step 1/64 or 1/128 (Section 4.3)")
    ap.add_argument("--sweep-phi", type=int, choices=(1, 2), default=1,
                    help="sweep: Matern parameter set Phi_1 (isotropic) or Phi_2 (anisotropic) of Table Matern")
    ap.add_argument("--eps-sweep", action="store_true",
                    help="pcmlmc gardner: cost of Algorithm 1 against the tolerance, the finest grid refined "
                         "as eps halves (h_L ~ eps)")
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--in-flight", type=int, default=2,
                    help="gardner/vg: steps kept in flight at once: as many library contexts, each driven "
                         "by a host thread of its own on a stream of its own, share the timed steps "
                         "(1: one step after another; the JSON line also reports that rate)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed calls first (the first calls of a workload tune tiles and the schedule: "
                         "default 9 for the batched MLMC calls, 5 otherwise)")
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    ap.add_argument("--max-picard", type=int, default=None,
                    help="Picard iterations per step, first attempt (default 100; adjoint workload 500)")
    ap.add_argument("--cycles", type=int, default=1, help="cycles per Picard iteration")
    ap.add_argument("--cycle", choices=("V", "W"), default="V")
    ap.add_argument("--fallback-cycles", type=int, default=None,
                    help="cycles per Picard step of the fallback attempt of a failed sample (0: none; default 2, "
                         "adjoint workload 0)")
    ap.add_argument("--fallback-max-picard", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--confine", choices=("default", "on", "off"), default="default",
                    help="confine the classes of the batched call to parts of the compute units (on: flag "
                         "bit 7, off: bit 8); default: the library's schedule tuner decides")
    ap.add_argument("--no-autotune", action="store_true",
                    help="32 x 32 streaming tiles on every level and no schedule tuning (profiling runs: "
                         "timing under a counter profiler is distorted)")
    ap.add_argument("--tune-cache", default="",
                    help="file for the library's tuning choices (read at start, written when it tunes), so "
                         "that a profiled run repeats an unprofiled run's tiles and schedule")
    ap.add_argument("--tiles", choices=("auto", "32", "16"), default="auto",
                    help="streaming tile edges: autotuned (default), or 32 / 16 on every level")
    ap.add_argument("--large-batch", action="store_true",
                    help="only the down-leg smoother's rate on the large batch (64 samples of 512^2)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-grid, FP64-path, solver-variant and large-batch figures (outside the "
                         "timed region)")
    args = ap.parse_args()
    # the adjoint workload keeps one attempt with a 500-iteration limit: with a 100-iteration
    # first attempt and the fallback, 639 of its 1024 samples got gradients, against 835
    adj = args.workload == "adjoint"
    if args.warmup is None:
        args.warmup = 9 if args.workload in ("gardner", "vg") else 5
    if args.max_picard is None:
        args.max_picard = 500 if adj else 100
    if args.fallback_cycles is None:
        args.fallback_cycles = 0 if adj else 2
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sample-parallel "
              "multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1903_08741_amd as rmg
    import workloads as W

    if args.workload == "adjoint":
        adjoint_bench(args, torch, rmg, W)
        return
    if args.workload == "sweep":
        sweep_bench(args, torch, rmg, W)
        return
    if args.workload == "kl":
        kl_bench(args, torch, rmg, W)
        return
    if args.workload == "pcmlmc":
        if args.eps_sweep:
            pcmlmc_eps_sweep(args, torch, rmg, W)
        else:
            pcmlmc_bench(args, torch, rmg, W)
        return
    dev = torch.device("cuda:0")
    precision = rmg.MIXED if args.precision == "mixed" else rmg.FP64
    vg = args.workload == "vg"
    build = build_vg_levels if vg else build_levels
    levels, opts, marg = build(torch, rmg, W, precision, dev, args.max_picard)
    opts.cycles_per_picard = args.cycles
    opts.cycle = rmg.CYCLE_W if args.cycle == "W" else rmg.CYCLE_V
    opts.fallback_cycles = args.fallback_cycles
    opts.fallback_max_picard = args.fallback_max_picard if args.fallback_cycles else 0
    if args.no_autotune or args.tiles == "32":
        opts.flags |= rmg.FLAG_NO_AUTOTUNE
    if args.tiles == "16":
        opts.flags |= rmg.FLAG_TILES_16
    if args.confine == "on":
        opts.flags |= rmg.FLAG_CONFINE
    elif args.confine == "off":
        opts.flags |= rmg.FLAG_NO_CONFINE
    ctx = rmg.Context(0, tune_cache=args.tune_cache) if args.tune_cache else rmg.default_context(0)
    if args.large_batch:
        print(json.dumps({"roofline_large_batch": large_batch_roofline(torch, rmg, ctx, W, levels, marg)}), flush=True)
        return
    if args.grid:
        res = per_grid(torch, rmg, ctx, levels, opts, marg, only=args.grid)
        if not res:
            sys.exit(f"no grid-size class {args.grid} in this workload")
        r = res[str(args.grid)]
        print(json.dumps({"metric": "Picard-MG sample solves/sec of one grid-size class", "value": r["solves_per_s"],
                          "unit": "sample solves/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": r["ms"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32 multigrid in f64 Picard" if precision == rmg.MIXED else "f64",
                          "data": "synthetic (seeded KL lognormal Ks fields)",
                          "config": {"workload": f"grid {args.grid} class of the {'vg' if vg else 'gardner'} MLMC "
                                                 f"workload", **r}}), flush=True)
        return
    total = n_solves(levels)
    sums = None
    for i in range(args.warmup):
        t0 = time.time()
        sums, _, rc = ctx.mlmc_level_estimate(levels, marg, opts)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.time() - t0:.3f}s rc={rc}")
    from paper_1903_08741_amd import _abi
    if args.in_flight < 1:
        sys.exit("--in-flight must be at least 1")
    ctxs = [ctx]
    fopts = opts
    if args.in_flight > 1:
        if args.confine == "default":
            # steps in flight run unconfined: the confined classes of two contexts take the
            # same compute-unit masks on queues of their own and did not overlap (340 against
            # 235 ms per step unconfined, the same results)
            fopts = rmg.SolverOpts(**{**opts.__dict__})
            fopts.flags |= rmg.FLAG_NO_CONFINE
            for i in range(args.warmup):  # the unconfined schedule's batch length
                ctx.mlmc_level_estimate(levels, marg, fopts)
            torch.cuda.synchronize()
        ctxs += extra_contexts(rmg, ctx, args.in_flight - 1, args.tune_cache)
        for j, c in enumerate(ctxs[1:], 1):
            for i in range(args.warmup):
                c.mlmc_level_estimate(levels, marg, fopts)
            torch.cuda.synchronize()
            log(f"context {j}: {args.warmup} warm-up calls done")
    timed_kinds = _abi.TIME_SMOOTHER_DOWN | _abi.TIME_COARSE | _abi.TIME_FINE
    if args.in_flight == 1:
        ctx.set_kernel_timing(timed_kinds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.in_flight > 1:
        runs = run_in_flight(torch, ctxs, args.steps,
                             lambda c: c.mlmc_level_estimate(levels, marg, fopts, return_qoi=True))
    else:
        runs = []
        for i in range(args.steps):
            runs.append(ctx.mlmc_level_estimate(levels, marg, opts, return_qoi=True))
            log(f"step {i} done rc={runs[-1][2]}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1000.0 * dt / args.steps
    sums = runs[-1][0]
    identical = same_results(torch, runs)
    if not identical:
        log("WARNING: the timed steps did not all return the same results")
    converged = sum(s["n"] * (2 if lv["n_coarse"] else 1) for s, lv in zip(sums, levels))
    sequential = None
    if args.in_flight > 1:
        # the per-kernel rates come from these sequential steps: with steps in flight a
        # launch's event pair also brackets its wait for compute units that the other
        # step's kernels hold (24 us per k_down launch with two steps fully overlapped,
        # against 6-7 us alone)
        for c in ctxs[1:]:
            c.close()
        ctx.set_kernel_timing(timed_kinds)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            ssums, _, _ = ctx.mlmc_level_estimate(levels, marg, opts)
        torch.cuda.synchronize()
        sms = 1e3 * (time.perf_counter() - t1) / args.steps
        sequential = {"ms_per_step": sms, "value": converged / (sms / 1e3), "steps": args.steps,
                      "same_level_sums": ssums == sums,
                      "note": "the same steps one after another on one context with the tuned schedule "
                              "(outside the timed region)"}
        log(f"sequential: {sms:.1f} ms per step")
    kt = ctx.kernel_timing(_abi.TIME_SMOOTHER_DOWN)
    schedule = tuned_schedule(ctx)
    kc = ctx.kernel_timing(_abi.TIME_COARSE)
    kf = ctx.kernel_timing(_abi.TIME_FINE)
    ctx.set_kernel_timing(_abi.TIME_NONE)
    per_level = level_report(sums, levels)
    for r in per_level:
        log(f"level {r['level']} ({r['grid']}^2): pairs {r['pairs']} failed {r['failed']} retried {r['retried']} "
            f"picard_its {r['picard_its']}")
    failed = sum(s["n_failed"] for s in sums)
    picard = sum(s["picard_its"] for s in sums)
    gbs = kt["algo_bytes"] / (kt["total_ms"] * 1e-3) / 1e9 if kt["total_ms"] > 0 else 0.0
    es = 4 if precision == rmg.MIXED else 8
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": None if vg else recorded_traffic(),
            "kernel": "k_down (nu1 fused red-black sweeps + residual + restriction, level-streaming path)",
            "timing": "kernel execution time: each timed launch's event pair is recorded by its dispatch"
                      + (" (over the sequential steps: see 'sequential')" if args.in_flight > 1 else ""),
            "launches": kt["launches"], "avg_launch_us": 1e3 * kt["total_ms"] / max(1, kt["launches"]),
            "algo_bytes_per_launch": kt["algo_bytes"] / max(1, kt["launches"]),
            "compulsory_bytes_per_cell": 5.25 * es,
            "sweep_model_bytes_per_cell": (2 * 20 + 17) * es / 4,
            "frac_sweep_model": (gbs * (2 * 20 + 17) / 4 / 5.25) / HBM_PEAK_GBS}
    tus = None if vg else recorded_trace_us()
    if tus and kt["launches"]:
        # the same algorithmic bytes per launch at the committed trace's average duration
        tg = roof["algo_bytes_per_launch"] / (tus * 1e-6) / 1e9
        roof.update({"traced_avg_launch_us": tus, "achieved_at_traced_us": tg, "frac_at_traced_us": tg / HBM_PEAK_GBS,
                     "event_over_trace": roof["avg_launch_us"] / tus})
    roof_fine = None
    if kf["total_ms"] > 0:
        fg = kf["algo_bytes"] / (kf["total_ms"] * 1e-3) / 1e9
        roof_fine = {"bound": "hbm", "kernel": "k_fine (FP64 outer residual, closure, level coefficients)",
                     "achieved": fg, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fg / HBM_PEAK_GBS,
                     "launches": kf["launches"], "avg_launch_us": 1e3 * kf["total_ms"] / kf["launches"],
                     "cells_per_s": kf["cells"] / (kf["total_ms"] * 1e-3)}
    extras = {}
    if not args.no_extras and not vg:
        extras["per_grid"] = per_grid(torch, rmg, ctx, levels, opts, marg)
        if precision == rmg.MIXED:
            fms, ffail = fp64_path(torch, rmg, ctx, levels, marg, opts)
            # against the mixed path's steps one at a time, as the FP64 path is timed
            ref_ms = sequential["ms_per_step"] if sequential else ms
            extras["fp64_path"] = {"ms_per_step": fms, "failed_pairs": ffail, "mixed_speedup": fms / ref_ms}
        extras["solver_variants"] = solver_variants(torch, rmg, ctx, levels, marg, opts, total)
        extras["roofline_large_batch"] = large_batch_roofline(torch, rmg, ctx, W, levels, marg)
    cpu = None
    if not args.no_cpu_baseline and not vg:
        t1 = time.time()
        cpu = cpu_baseline(dict(max_picard=args.max_picard, cycles_per_picard=args.cycles,
                                cycle=args.cycle, fallback_cycles=args.fallback_cycles,
                                fallback_max_picard=args.fallback_max_picard), converged=converged)
        log(f"cpu baseline {time.time() - t1:.1f}s")
    fb = (f", failed samples restarted with {args.fallback_cycles} {args.cycle}(2,2) per Picard step "
          f"(limit {args.fallback_max_picard})" if args.fallback_cycles else "")
    out = {
        "metric": METRIC,
        "value": converged / (ms / 1000.0),
        "unit": "sample solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 multigrid in f64 Picard" if precision == rmg.MIXED else "f64",
        "data": ("synthetic (seeded KL fields: lognormal Ks, alpha, 1 + lognormal n)" if vg
                 else "synthetic (seeded KL lognormal Ks fields)"),
        "config": {"workload": ("mlmc 5 levels 32^2..512^2, 2048/512/128/32/8 samples, van Genuchten-Mualem "
                                "with 3 KL fields (128 modes), infiltration problem (eq. travellingwave, "
                                "Ks_bl 0.2), n shifted by (L-l)*0.1, 50 steps dt=0.005, "
                                f"{args.cycle}(2,2) x{args.cycles} per Picard, eps 1e-8" if vg else
                                "mlmc 5 levels 16^2..256^2, 4096/1024/256/64/16 samples, Gardner, "
                                f"10 steps dt=0.01, {args.cycle}(2,2) x{args.cycles} per Picard, eps 1e-8, "
                                f"limit {args.max_picard}") + fb,
                   "solves_per_step": total, "converged_solves_per_step": converged,
                   "cells_per_step": sum(lv["xi"].shape[0] * (lv["n_fine"] ** 2 + lv["n_coarse"] ** 2)
                                         for lv in levels),
                   "failed_pairs": failed, "retried_pairs": sum(s["n_retried"] for s in sums),
                   "levels": per_level,
                   "picard_iterations_per_step": picard, "precision": args.precision,
                   "cycles_per_picard": args.cycles, "max_picard": args.max_picard,
                   "fallback_cycles": args.fallback_cycles, "confine": args.confine, "schedule": schedule,
                   "steps_in_flight": args.in_flight,
                   "in_flight_confine": ("off" if fopts is not opts else args.confine) if args.in_flight > 1 else None},
        "in_flight_results_identical": identical,
        "sequential": sequential,
        "roofline": roof,
        "roofline_coarse": coarse_bound(kc),
        "roofline_fine": roof_fine,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
