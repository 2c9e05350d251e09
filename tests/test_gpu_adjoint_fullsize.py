"""Adjoint at the full size of its workload, in the benchmark's launch configuration.

1024 samples of 128^2, Gardner, 100 KL coefficients, 20 steps of dt = 0.01,
forward to 1e-8 with one V(2,2) per Picard step (at most 500 per step),
checkpoints every 5 steps, mixed precision, adjoint to 1e-13 (absolute; the
multipliers are ~1e-4 here).  The oracle
cannot run 1024 adjoints in a test, so:
  - sampled outputs: one converged sample against the oracle adjoint (twin
    forward, sparse-LU adjoint): Q within 1e-8, dQ/dxi within 1e-6 of its max;
    one failed sample fails in the oracle too;
  - properties at any size: checkpointing every 5 steps equals storing every step
    bit for bit; the mixed path's gradients equal the FP64 path's within 1e-7;
  - finite differences in the same configuration: 8 coefficients of one sample
    (17 samples of the same grid, forward and adjoint in FP64 to 1e-13), within
    1e-5 relative.
"""
from __future__ import annotations

import functools

import numpy as np
import pytest
import torch

import paper_1903_08741_amd as rmg
import workloads as W
from oracle import adjoint as oadj, kl as okl
from gpu_common import say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
CFG = W.ADJOINT_128
N, S, M, STEPS = CFG["n"], CFG["n_samples"], CFG["n_modes"], CFG["n_steps"]
MARG = (0.0, W.KS_FIELD["log_mean"], W.KS_FIELD["scale"])


@functools.lru_cache(maxsize=None)
def basis():
    f = W.KS_FIELD
    _, B = okl.basis(f["sigma2"], f["corr_len"], M, [N], ref_n=64)
    return B[N]


def prob():
    g = W.GARDNER_INFILTRATION
    return rmg.Problem(model=rmg.GARDNER, n_steps=STEPS, theta_r=g["theta_r"], theta_s=g["theta_s"],
                       gardner_a=g["gardner_a"], h_top=g["h_top"], h_bottom=g["h_bottom"], h_init=g["h_init"],
                       dt=g["dt"])


def xi_all():
    return W.xi_draws(CFG["workload_id"], 0, range(S), 1, M)[:, 0, :].copy()


def call(xi, precision=rmg.MIXED, ckpt=CFG["ckpt_every"], eps_picard=1e-8, max_picard=500, eps_adj=1e-13):
    B = torch.from_numpy(basis()).to(DEV)
    x = torch.from_numpy(np.ascontiguousarray(xi)).to(DEV)
    out = rmg.picard_mg_adjoint(N, B, x, MARG, prob(),
                                rmg.SolverOpts(precision=precision, eps_picard=eps_picard, max_picard=max_picard),
                                ckpt_every=ckpt, eps_adjoint=eps_adj)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in out.items()}


@pytest.fixture(scope="module")
def runs():
    xi = xi_all()
    out = {}
    for name, kw in (("mixed", {}), ("mixed_ckpt1", {"ckpt": 1}), ("fp64", {"precision": rmg.FP64})):
        say(f"full-size adjoint run: {name}")
        out[name] = call(xi, **kw)
    return out


def _oracle(i, max_picard=500):
    xi = xi_all()[i]
    B = basis()
    Ks = okl.lognormal(okl.gaussian_field(xi, B), MARG[1], MARG[2]).reshape(N, N)
    say(f"oracle adjoint of sample {i}")
    return oadj.solve_with_gradient(dict(W.GARDNER_INFILTRATION, n_steps=STEPS), Ks, N,
                                    dict(W.SOLVER, max_picard=max_picard), basis=B, marginal=MARG, mode="mg")


def test_full_size_checkpointing_is_bit_identical(runs):
    a, b = runs["mixed"], runs["mixed_ckpt1"]
    assert np.array_equal(a["status"], b["status"])
    assert np.array_equal(a["q"], b["q"], equal_nan=True)
    assert np.array_equal(a["grad"], b["grad"], equal_nan=True)


def test_full_size_mixed_matches_fp64(runs):
    a, b = runs["mixed"], runs["fp64"]
    ok = (a["status"] == 0) & (b["status"] == 0)
    assert ok.sum() > S // 2
    rel = np.max(np.abs(a["grad"][ok] - b["grad"][ok]), axis=1) / np.max(np.abs(b["grad"][ok]), axis=1)
    assert rel.max() <= 1e-7, rel.max()
    assert np.max(np.abs(a["q"][ok] - b["q"][ok]) / np.abs(b["q"][ok])) <= 1e-8


def test_full_size_converged_sample_matches_oracle(runs):
    a = runs["mixed"]
    i = int(np.flatnonzero(a["status"] == 0)[0])
    r = _oracle(i)
    assert r["status"] == 0
    assert abs(a["q"][i] - r["Q"]) <= 1e-8 * abs(r["Q"])
    assert np.max(np.abs(a["grad"][i] - r["dQ_dxi"])) <= 1e-6 * np.max(np.abs(r["dQ_dxi"]))


def test_full_size_failed_sample_fails_in_oracle(runs):
    a = runs["mixed"]
    bad = np.flatnonzero(a["status"] != 0)
    if bad.size == 0:
        pytest.skip("no failed sample in this workload")
    i = int(bad[0])
    assert np.isnan(a["q"][i]) and np.isnan(a["grad"][i]).all()
    assert _oracle(i)["status"] != 0


def test_full_size_gradient_matches_central_differences(runs):
    a = runs["fp64"]
    i = int(np.flatnonzero(a["status"] == 0)[0])
    x0 = xi_all()[i]
    e = 1e-6
    X = np.repeat(x0[None, :], 17, axis=0)
    for j in range(8):
        X[1 + 2 * j, j] += e
        X[2 + 2 * j, j] -= e
    say(f"finite differences on sample {i}, 8 coefficients")
    r = call(X, precision=rmg.FP64, eps_picard=1e-13, max_picard=3000, eps_adj=1e-13)
    assert (r["status"] == 0).all()
    g = r["grad"][0]
    fd = (r["q"][1::2] - r["q"][2::2]) / (2 * e)
    for j in range(8):
        assert abs(fd[j] - g[j]) <= 1e-5 * max(abs(fd[j]), 1e-3 * np.max(np.abs(g))), (j, fd[j], g[j])
