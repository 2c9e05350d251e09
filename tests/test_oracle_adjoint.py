"""Pins of the oracle's discrete adjoint (oracle/adjoint.py) against finite
differences of the forward model, which fixes what the derivative must be.

  - the assembled Jacobian dR/dp equals central differences of the step residual;
  - the derivative of R in log Ks equals central differences;
  - dQ/dxi of the whole time integration equals central differences of Q with the
    forward solved to 1e-13 by sparse LU (eps = 1e-6 on the KL coefficients),
    within 1e-5 relative (the tolerance fixed for gradients), for Gardner and for
    the linear law (whose K does not depend on p, so dK/dp terms vanish).
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, constitutive, kl

N_GRID = 8


def _prob(model="gardner", n_steps=4):
    if model == "linear":
        return dict(model="linear", theta_r=0.05, theta_s=0.5, c0=0.02, h_top=0.0, h_bottom=-2.0, h_init=-2.0,
                    dt=0.01, n_steps=n_steps)
    return dict(W.GARDNER_INFILTRATION, n_steps=n_steps)


def _fields(seed=3, n=N_GRID, M=6):
    _, B = kl.basis(1.0, 0.3, M, [n], ref_n=16)
    xi = W.normal_array([seed], (M,))
    Ks = kl.lognormal(kl.gaussian_field(xi, B[n]), 0.0, 1.0).reshape(n, n)
    return B[n], xi, Ks


def test_jacobian_matches_central_differences():
    prob = _prob()
    _, _, Ks = _fields()
    fields = {"Ks": Ks}
    p = -1.0 - 3.0 * W.uniform_array([9], (N_GRID, N_GRID))
    p[3, 4] = 0.2  # one saturated cell
    _, th_old, _ = constitutive.evaluate(prob, p - 0.1, fields)
    J = adjoint.jacobian(prob, fields, p).toarray()
    e = 1e-6
    for c in range(N_GRID * N_GRID):
        dp = np.zeros(N_GRID * N_GRID)
        dp[c] = e
        fd = (adjoint.residual(prob, fields, p + dp.reshape(p.shape), th_old)
              - adjoint.residual(prob, fields, p - dp.reshape(p.shape), th_old)) / (2 * e)
        scale = np.max(np.abs(J[:, c]))
        assert np.max(np.abs(fd - J[:, c])) <= 1e-6 * scale, c


def test_log_ks_derivative_matches_central_differences():
    prob = _prob()
    _, _, Ks = _fields()
    p = -1.0 - 3.0 * W.uniform_array([10], (N_GRID, N_GRID))
    _, th_old, _ = constitutive.evaluate(prob, p - 0.1, {"Ks": Ks})
    K, _, _ = constitutive.evaluate(prob, p, {"Ks": Ks})
    E = adjoint.flux_derivative(prob, p, K, K).toarray()
    e = 1e-6
    for c in range(0, N_GRID * N_GRID, 5):
        up, dn = Ks.copy(), Ks.copy()
        up.ravel()[c] *= np.exp(e)
        dn.ravel()[c] *= np.exp(-e)
        fd = (adjoint.residual(prob, {"Ks": up}, p, th_old) - adjoint.residual(prob, {"Ks": dn}, p, th_old)) / (2 * e)
        assert np.max(np.abs(fd - E[:, c])) <= 1e-6 * np.max(np.abs(E[:, c])), c


@pytest.mark.parametrize("model", ["gardner", "linear"])
def test_gradient_matches_central_differences_of_q(model):
    prob = _prob(model)
    B, xi, Ks = _fields()
    opts = dict(W.SOLVER, eps_picard=1e-13, max_picard=200)
    marg = (0.0, 0.0, 1.0)
    r = adjoint.solve_with_gradient(prob, Ks, N_GRID, opts, basis=B, marginal=marg, mode="direct")
    assert r["status"] == 0

    def q_of(x):
        K = kl.lognormal(kl.gaussian_field(x, B), 0.0, 1.0).reshape(N_GRID, N_GRID)
        out = adjoint.solve_with_gradient(prob, K, N_GRID, opts, mode="direct")
        return out["Q"]

    e = 1e-6
    for j in range(B.shape[0]):
        d = np.zeros_like(xi)
        d[j] = e
        fd = (q_of(xi + d) - q_of(xi - d)) / (2 * e)
        assert abs(fd - r["dQ_dxi"][j]) <= 1e-5 * max(abs(fd), 1e-3 * np.max(np.abs(r["dQ_dxi"]))), (j, fd,
                                                                                                  r["dQ_dxi"][j])
