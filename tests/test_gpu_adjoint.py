"""GPU parity of the discrete adjoint (picard_mg_adjoint, outflux_qoi).

Gardner infiltration (a = 1, h0 = -10, top 0, bottom -10), Ks = exp(G) from the
KL expansion of the exponential covariance (correlation length 0.3), the
quantity Q = time-integrated bottom outflux.  Checks:
  - against the oracle adjoint (exact Jacobians, sparse LU) on the twin forward
    iteration: Q within 1e-10 and dQ/dxi within 1e-7 of max |dQ/dxi| (FP64);
  - against central finite differences of the GPU's own Q (eps = 1e-6 on eight
    KL coefficients, forward converged to 1e-13): within 1e-5 relative, the
    tolerance fixed for gradients;
  - checkpointing (recomputed segments) gives bit-identical results to storing
    every step; the mixed-precision adjoint matches the FP64 one;
  - the torch.autograd.Function returns the adjoint gradient; a failed forward
    sample reports its status and NaN outputs.
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
MARG = (0.0, 0.0, 1.0)


@functools.lru_cache(maxsize=None)
def basis(M, grids=(8, 16, 64, 128)):
    _, B = okl.basis(1.0, 0.3, M, list(grids), ref_n=32)
    return B


def gprob(n_steps):
    g = W.GARDNER_INFILTRATION
    return rmg.Problem(model=rmg.GARDNER, n_steps=n_steps, theta_r=g["theta_r"], theta_s=g["theta_s"],
                       gardner_a=g["gardner_a"], h_top=g["h_top"], h_bottom=g["h_bottom"], h_init=g["h_init"],
                       dt=g["dt"])


def oprob(n_steps):
    return dict(W.GARDNER_INFILTRATION, n_steps=n_steps)


def run(n, xi, M, n_steps, precision=rmg.FP64, eps_picard=1e-12, ckpt=1, max_picard=1000, eps_adj=1e-13):
    B = torch.from_numpy(basis(M)[n]).to(DEV)
    x = torch.from_numpy(np.ascontiguousarray(xi)).to(DEV)
    out = rmg.picard_mg_adjoint(n, B, x, MARG, gprob(n_steps),
                                rmg.SolverOpts(precision=precision, eps_picard=eps_picard, max_picard=max_picard),
                                ckpt_every=ckpt, eps_adjoint=eps_adj)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("n,S,M,n_steps", [(8, 3, 6, 4), (16, 2, 8, 4), (64, 1, 8, 3), (128, 1, 8, 2)])
def test_adjoint_matches_oracle_adjoint(n, S, M, n_steps):
    xi = W.normal_array([21, n], (S, M))
    say(f"adjoint vs oracle n={n} S={S} M={M} steps={n_steps}")
    out = run(n, xi, M, n_steps)
    assert out["rc"] == 0
    q, g = out["q"].cpu().numpy(), out["grad"].cpu().numpy()
    B = basis(M)[n]
    opts = dict(W.SOLVER, eps_picard=1e-12, max_picard=1000)
    for s in range(S):
        Ks = okl.lognormal(okl.gaussian_field(xi[s], B), 0.0, 1.0).reshape(n, n)
        r = oadj.solve_with_gradient(oprob(n_steps), Ks, n, opts, basis=B, marginal=MARG, mode="mg")
        assert r["status"] == 0
        assert abs(q[s] - r["Q"]) <= 1e-10 * abs(r["Q"]), (s, q[s], r["Q"])
        scale = np.max(np.abs(r["dQ_dxi"]))
        assert np.max(np.abs(g[s] - r["dQ_dxi"])) <= 1e-7 * scale, (s, g[s], r["dQ_dxi"])


def test_adjoint_matches_central_differences():
    n, M, n_steps = 16, 8, 4
    xi = W.normal_array([22], (1, M))
    say("adjoint vs central differences n=16")
    base = run(n, xi, M, n_steps, eps_picard=1e-13, max_picard=3000)
    assert base["rc"] == 0
    g = base["grad"].cpu().numpy()[0]
    e = 1e-6
    X = np.repeat(xi, 2 * M, axis=0)
    for j in range(M):
        X[2 * j, j] += e
        X[2 * j + 1, j] -= e
    pert = run(n, X, M, n_steps, eps_picard=1e-13, max_picard=3000)
    assert pert["rc"] == 0
    qp = pert["q"].cpu().numpy()
    fd = (qp[0::2] - qp[1::2]) / (2 * e)
    for j in range(M):
        assert abs(fd[j] - g[j]) <= 1e-5 * max(abs(fd[j]), 1e-3 * np.max(np.abs(fd))), (j, fd[j], g[j])


@pytest.mark.parametrize("n", [16, 64])
def test_checkpointed_segments_are_bit_identical(n):
    M, n_steps = 8, 4
    xi = W.normal_array([23, n], (3, M))
    say(f"checkpoint segments n={n}")
    a = run(n, xi, M, n_steps, ckpt=1)
    b = run(n, xi, M, n_steps, ckpt=2)
    assert torch.equal(a["q"], b["q"]) and torch.equal(a["grad"], b["grad"])


@pytest.mark.parametrize("n", [16, 64])
def test_mixed_precision_adjoint_matches_fp64(n):
    M, n_steps = 8, 3
    xi = W.normal_array([24, n], (2, M))
    say(f"mixed adjoint n={n}")
    a = run(n, xi, M, n_steps)
    b = run(n, xi, M, n_steps, precision=rmg.MIXED, eps_adj=1e-11)
    assert a["rc"] == 0 and b["rc"] == 0
    ga, gb = a["grad"].cpu().numpy(), b["grad"].cpu().numpy()
    assert np.max(np.abs(ga - gb)) <= 1e-6 * np.max(np.abs(ga))
    assert np.max(np.abs(a["q"].cpu().numpy() - b["q"].cpu().numpy())) <= 1e-8 * np.max(np.abs(a["q"].cpu().numpy()))


def test_autograd_function_returns_the_adjoint_gradient():
    n, M, n_steps = 8, 6, 3
    xi = torch.from_numpy(W.normal_array([25], (4, M))).to(DEV).requires_grad_(True)
    B = torch.from_numpy(basis(M)[n]).to(DEV)
    opts = rmg.SolverOpts(precision=rmg.FP64, eps_picard=1e-12, max_picard=1000)
    q = rmg.outflux_qoi(xi, B, n, MARG, gprob(n_steps), opts)
    w = torch.arange(1, 5, dtype=torch.float64, device=DEV)
    (q * w).sum().backward()
    ref = rmg.picard_mg_adjoint(n, B, xi.detach(), MARG, gprob(n_steps), opts)
    assert torch.equal(q.detach(), ref["q"])
    assert torch.equal(xi.grad, w[:, None] * ref["grad"])


def test_failed_forward_sample_is_reported():
    n, M = 16, 6
    xi = W.normal_array([26], (2, M))
    out = run(n, xi, M, 2, eps_picard=1e-12, max_picard=2)
    assert out["rc"] == rmg.RMG_ENOTCONV
    st = out["status"].cpu().numpy()
    assert (st == rmg.SAMPLE_MAXITER).all()
    assert torch.isnan(out["q"]).all() and torch.isnan(out["grad"]).all()


def test_invalid_adjoint_arguments_raise():
    n, M = 8, 6
    xi = torch.from_numpy(W.normal_array([27], (1, M))).to(DEV)
    B = torch.from_numpy(basis(M)[n]).to(DEV)
    with pytest.raises(rmg.RmgError):
        rmg.picard_mg_adjoint(n, B, xi, MARG, gprob(3), rmg.SolverOpts(), ckpt_every=2)
    with pytest.raises(rmg.RmgError):
        rmg.picard_mg_adjoint(n, B, xi, MARG, rmg.Problem(model=rmg.VGM), rmg.SolverOpts())


@pytest.mark.parametrize("precision", [rmg.FP64, rmg.MIXED])
def test_forward_only_outflux_equals_the_adjoints_q(precision):
    """picard_mg_outflux (the autograd Function's forward pass: the forward solve alone)
    returns the same Q as picard_mg_adjoint, bit for bit, with and without checkpoints."""
    n, M, n_steps = 64, 6, 4
    xi = torch.from_numpy(W.normal_array([27], (5, M))).to(DEV)
    B = torch.from_numpy(basis(M)[n]).to(DEV)
    opts = rmg.SolverOpts(precision=precision, max_picard=300)
    ctx = rmg.default_context()
    fwd = ctx.picard_mg_outflux(n, B, xi, MARG, gprob(n_steps), opts)
    for ck in (1, 2):
        ref = rmg.picard_mg_adjoint(n, B, xi, MARG, gprob(n_steps), opts, ckpt_every=ck)
        assert torch.equal(fwd["q"], ref["q"]), ck
        assert torch.equal(fwd["status"], ref["status"])
    with torch.no_grad():
        q = rmg.outflux_qoi(xi, B, n, MARG, gprob(n_steps), opts)
    assert torch.equal(q, fwd["q"])
