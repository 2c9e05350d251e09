"""GPU parity of the adaptive PC_MLMC driver (Section 5.1, Algorithm 1).

Hierarchy: grids 4^2, 8^2, 16^2 (a pair of level l couples 2^(l+2) with 2^(l+1)),
Gardner closure with the exponent a as the continuation parameter (0.5, 0.75 and
1.0 from the coarsest to the finest level: milder nonlinearity below), 4 time
steps, FP64 (the oracle's own iteration, so cycle counts and failure decisions
coincide), cost in work units (cycles x cells).  The oracle runs Algorithm 1 with
its own solver on the same seeded draws; the two must take the same decisions
(rounds, pairs drawn, targets, cost per pair) and agree on the estimates.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1903_08741_amd as rmg
import workloads as W
from oracle import mlmc as omlmc, pc_mlmc as opc
from gpu_common import oracle_basis, oracle_fields, oracle_solve, say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
WID = 77
GRIDS = [(4, 0), (8, 4), (16, 8)]
A = [0.5, 0.75, 1.0]
WARM = [8, 4, 4]
EPS = 2e-2
N_STEPS = 4
MARG = [(0.0, W.KS_FIELD["log_mean"], W.KS_FIELD["scale"])]


def _oprob(l):
    return dict(W.GARDNER_INFILTRATION, gardner_a=A[l], n_steps=N_STEPS)


def _gprob(l):
    g = W.GARDNER_INFILTRATION
    return rmg.Problem(model=rmg.GARDNER, n_steps=N_STEPS, theta_r=g["theta_r"], theta_s=g["theta_s"],
                       gardner_a=A[l], h_top=g["h_top"], h_bottom=g["h_bottom"], h_init=g["h_init"], dt=g["dt"])


def _levels(B):
    out = []
    for l, (nf, nc) in enumerate(GRIDS):
        out.append(dict(n_fine=nf, n_coarse=nc, n_warmup=WARM[l], fine=_gprob(l),
                        coarse=_gprob(l - 1) if l else None,
                        basis_fine=torch.from_numpy(B[nf]).to(DEV),
                        basis_coarse=torch.from_numpy(B[nc]).to(DEV) if l else None))
    return out


class Source:
    """Seeded draws; records every request to check the numbering."""

    def __init__(self):
        self.calls = []

    def __call__(self, level, first, count):
        self.calls.append((level, first, count))
        return W.xi_draws(WID, level, range(first, first + count), 1, W.KS_FIELD["n_modes"])


@pytest.fixture(scope="module")
def oracle_run():
    B = oracle_basis()
    opts = dict(W.SOLVER, max_picard=100)

    def sample(l, i):
        xi = W.xi_draws(WID, l, [i], 1, W.KS_FIELD["n_modes"])[0, 0]
        nf, nc = GRIDS[l]
        rf = oracle_solve(nf, oracle_fields(B[nf], xi), _oprob(l), opts)
        if not l:
            return rf["qoi"], None, rf["cycles"], 0
        rc = oracle_solve(nc, oracle_fields(B[nc], xi), _oprob(l - 1), opts)
        return rf["qoi"], rc["qoi"], rf["cycles"], rc["cycles"]

    def bias_pair(i):
        # the finest level's pair i with its own parameter set on both grids (eq. numErr)
        L = len(GRIDS) - 1
        xi = W.xi_draws(WID, L, [i], 1, W.KS_FIELD["n_modes"])[0, 0]
        nf, nc = GRIDS[L]
        return (oracle_solve(nf, oracle_fields(B[nf], xi), _oprob(L), opts)["qoi"],
                oracle_solve(nc, oracle_fields(B[nc], xi), _oprob(L), opts)["qoi"])

    say("oracle PC_MLMC run")
    return opc.run(sample, GRIDS, WARM, EPS, bias_pair=bias_pair)


def _run(cap, cost=rmg.COST_WORK, precision=rmg.FP64):
    src = Source()
    say(f"GPU PC_MLMC run: max_pairs_per_call={cap} cost_model={cost} precision={precision}")
    r = rmg.pc_mlmc(_levels(oracle_basis()), MARG, rmg.SolverOpts(precision=precision, max_picard=100), EPS, src,
                    cost_model=cost, max_pairs_per_call=cap)
    return r, src


@pytest.fixture(scope="module")
def gpu_runs():
    return {cap: _run(cap) for cap in (5, 0)}


@pytest.mark.parametrize("cap", [5, 0])
def test_pc_mlmc_takes_the_oracles_decisions(oracle_run, gpu_runs, cap):
    r, _ = gpu_runs[cap]
    o = oracle_run
    assert r["rc"] == rmg.RMG_OK and r["converged"] == 1 and o["converged"]
    assert r["rounds"] == o["rounds"]
    for g, x in zip(r["levels"], o["levels"]):
        assert g["drawn"] == x["drawn"] and g["target"] == x["target"]
        assert g["sums"]["n"] == x["sums"]["n"] and g["sums"]["n_failed"] == x["sums"]["n_failed"]
        assert g["W"] == x["W"]
        assert abs(g["V"] - x["V"]) <= 1e-8 * x["V"] + 1e-15
        assert abs(g["mean"] - x["mean"]) <= 1e-10
    assert abs(r["mean"] - o["mean"]) <= 1e-10
    assert abs(r["var"] - o["var"]) <= 1e-9 * abs(o["var"])
    assert abs(r["sampling_err2"] - o["sampling_err2"]) <= 1e-8 * o["sampling_err2"]
    assert r["sampling_err2"] <= EPS ** 2
    assert r["bias_pairs"] == o["bias_pairs"] > 0
    assert abs(r["bias"] - o["bias"]) <= 1e-8 * o["bias"]


def test_pc_mlmc_draw_numbering_and_batching(gpu_runs):
    for cap, (r, src) in gpu_runs.items():
        nxt = [0] * len(GRIDS)
        for level, first, count in src.calls:
            assert first == nxt[level] and count >= 1
            if cap:
                assert count <= cap
            nxt[level] += count
        # the bias pairs continue the finest level's numbering
        assert nxt == [x["drawn"] + (r["bias_pairs"] if l == len(GRIDS) - 1 else 0)
                       for l, x in enumerate(r["levels"])]


def test_pc_mlmc_sums_are_the_sums_of_the_drawn_pairs(gpu_runs):
    """Re-solve exactly the drawn pairs in one batched call: its sums (a different
    batching) agree with the driver's accumulated sums to rounding."""
    r, _ = gpu_runs[0]
    B = oracle_basis()
    levels = []
    for l, (lv, x) in enumerate(zip(_levels(B), r["levels"])):
        xi = torch.from_numpy(W.xi_draws(WID, l, range(x["drawn"]), 1, W.KS_FIELD["n_modes"])).to(DEV)
        levels.append(dict(lv, xi=xi))
    sums, q, _ = rmg.mlmc_level_estimate(levels, MARG, rmg.SolverOpts(precision=rmg.FP64, max_picard=100),
                                         return_qoi=True)
    for s, x in zip(sums, r["levels"]):
        for k in ("n", "n_failed", "picard_its", "mg_cycles", "mg_cycles_coarse"):
            assert s[k] == x["sums"][k], k
        for k in ("sY", "sY2", "sQf", "sQf2"):
            a, b = sum(s[k]), sum(x["sums"][k])
            assert abs(a - b) <= 4 * np.spacing(abs(b)), k


def test_pc_mlmc_time_cost_model_is_consistent():
    r, _ = _run(0, cost=rmg.COST_TIME)
    assert r["converged"] == 1 and all(x["W"] > 0 for x in r["levels"])
    N = omlmc.optimal_samples(EPS, [x["V"] for x in r["levels"]], [x["W"] for x in r["levels"]])
    for x, n in zip(r["levels"], N):
        assert x["target"] == max(int(n), 2) and x["sums"]["n"] >= x["target"]
    assert r["sampling_err2"] <= EPS ** 2


def test_pc_mlmc_mixed_precision_converges():
    r, _ = _run(0, precision=rmg.MIXED)
    assert r["converged"] == 1 and r["sampling_err2"] <= EPS ** 2


def test_pc_mlmc_rejects_a_broken_telescope():
    levels = _levels(oracle_basis())
    levels[2]["coarse"] = _gprob(2)  # should be level 1's fine problem
    with pytest.raises(rmg.RmgError, match="coarse problem differs"):
        rmg.pc_mlmc(levels, MARG, rmg.SolverOpts(precision=rmg.FP64), EPS, Source())
