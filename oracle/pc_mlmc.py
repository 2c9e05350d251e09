"""Adaptive multilevel Monte Carlo with parametric continuation (oracle, FP64).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

Section 5.1, Algorithm 1 (PC_MLMC), in the paper's order:
  1. fix the tolerance eps, the hierarchy (grid, time grid and parameter set
     Theta_l of every level) and the warm-up pair counts N*_l;
  2. estimate the level means (eq. SMC) and level variances (eq. level_var)
     from N*_l pairs on every level;
  3. set N_l by eq. MLMCSAMP;
  4. compute the additional pairs and update the estimates;
  5. repeat 3-4 until no level needs more pairs.
The cost per pair W_l is estimated from the warm-up pairs (the remark after
Algorithm 1).  With N_l >= the real-valued optimum of eq. MLMCSAMP the sampling
error sum_l V_l / N_l (eq. MLMCVar) is at most eps^2 (eq. errMLMC).

Readings where the paper is silent:
  - a failed pair (a member exceeded its Picard limit) enters no sum and is
    replaced by a new draw; N_l counts successful pairs and pair numbers are
    never reused, so the pairs of level l are numbers 0 .. drawn_l - 1;
  - N_l is at least 2, the fewest values a sample variance needs;
  - W_l in work units is multigrid cycles times cells of both members of a pair
    (Section 4.3 measures cost in cycles), over the pairs drawn in the warm-up
    (failed pairs included: their work was spent);
  - the bias estimate applies eq. discErr with mesh ratio s = 2 to the finest grid
    and the next coarser one under the same parameter set Theta_L (eq. numErr fixes
    Theta_L): sqrt(mean of (Q_{h_L} - Q_{h_{L-1}})^2) / (2^a - 1), the scalar-QoI form
    of its L2(Omega; D) norm.  With continuation the finest level's own pairs compare
    Theta_L with Theta_{L-1}, so max(2, N_L) further pairs of the finest level (numbers
    continuing its numbering, failed ones replaced) are solved with Theta_L on both
    grids; without continuation at the top the level's own pairs serve.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlmc


def run(sample_pair, grids, warmup, eps, bias_rate=1.0, max_rounds=50, max_pairs=1 << 40, bias_pair=None):
    """Algorithm 1.

    sample_pair(level, i) -> (q_fine, q_coarse, cycles_fine, cycles_coarse) for pair i of
        `level`: q_* are the QoIs of the two members (q_coarse None on level 0, NaN for a
        failed solve), cycles_* their multigrid cycle counts.
    grids: [(n_fine, n_coarse)] per level, n_coarse = 0 on level 0.
    warmup: N*_l per level.
    bias_pair(i) -> (q_fine, q_coarse) of pair i of the finest level with the finest
        level's parameter set on both grids; None when the hierarchy has no continuation
        at the top (the finest level's pairs then serve for the bias).
    Returns dict(levels=[dict(drawn, target, W, V, mean, sums, q_fine, q_coarse)], mean,
    var, sampling_err2, bias, bias_pairs, rounds, converged).
    """
    L = len(grids)
    qf = [[] for _ in range(L)]
    qc = [[] for _ in range(L)]
    work = [0] * L
    drawn = [0] * L

    def sums(l):
        return mlmc.level_sums(qf[l], qc[l] if l else None)

    def n_ok(l):
        return sums(l)["n"]

    def draw_until(l, target):
        while n_ok(l) < target and drawn[l] < max_pairs:
            a, b, cf, cc = sample_pair(l, drawn[l])
            qf[l].append(a)
            if l:
                qc[l].append(b)
            nf, nc = grids[l]
            work[l] += cf * nf * nf + cc * nc * nc
            drawn[l] += 1

    # step 2: warm-up pairs on every level, and W_l from them
    for l in range(L):
        draw_until(l, warmup[l])
    for l in range(L):
        if n_ok(l) < 2:
            raise RuntimeError(f"level {l}: fewer than two successful warm-up pairs")
    W = [work[l] / drawn[l] for l in range(L)]

    # steps 3-5
    target = list(warmup)
    rounds, converged, exhausted = 0, False, False
    while rounds < max_rounds:
        V = [max(0.0, mlmc.mc_var(sums(l))) for l in range(L)]
        N = mlmc.optimal_samples(eps, V, W)
        target = [max(int(x), 2) for x in N]
        rounds += 1
        if all(n_ok(l) >= target[l] for l in range(L)):
            converged = True
            break
        if exhausted:
            break
        for l in range(L):
            draw_until(l, target[l])
        exhausted = any(n_ok(l) < target[l] and drawn[l] >= max_pairs for l in range(L))

    S = [sums(l) for l in range(L)]
    est = mlmc.combine(S)
    V = [max(0.0, v) for v in est["level_var"]]
    err2 = math.fsum(V[l] / S[l]["n"] for l in range(L))
    bias, nb = float("nan"), 0
    if L > 1:
        sb = S[-1]
        if bias_pair is not None:
            bf, bc = [], []
            want = max(2, target[-1])
            while mlmc.level_sums(bf, bc)["n"] < want and drawn[-1] + nb < max_pairs:
                a, b = bias_pair(drawn[-1] + nb)
                bf.append(a)
                bc.append(b)
                nb += 1
            sb = mlmc.level_sums(bf, bc)
        if sb["n"]:
            bias = math.sqrt(sb["sY2"] / sb["n"]) / (2.0 ** bias_rate - 1.0)
    levels = [dict(drawn=drawn[l], target=target[l], W=W[l], V=V[l], mean=mlmc.mc_mean(S[l]), sums=S[l],
                   q_fine=np.array(qf[l]), q_coarse=np.array(qc[l]) if l else None) for l in range(L)]
    return dict(levels=levels, mean=est["mean"], var=est["var"], sampling_err2=err2, bias=bias, bias_pairs=nb,
                rounds=rounds, converged=converged and err2 <= eps * eps * (1 + 1e-12))
