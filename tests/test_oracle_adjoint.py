"""Pins of the oracle's discrete adjoint (oracle/adjoint.py) against finite
differences of the forward model, which fixes what the derivative must be.

  - the assembled Jacobian dR/dp equals central differences of the step residual;
  - the derivative of R in log Ks equals central differences;
  - dQ/dxi of the whole time integration equals central differences of Q with the
    forward solved to 1e-13 by sparse LU (eps = 1e-6 on the KL coefficients),
    within 1e-5 relative (the tolerance fixed for gradients), for Gardner and for
    the linear law (whose K does not depend on p, so dK/dp terms vanish);
  - dQ/dxi equals the complex-step derivative Im Q(xi + i t e_j) / t (t = 1e-30) of
    the forward model integrated in complex arithmetic, exact to rounding (no
    cancellation), within 1e-11 relative on 8^2 and 16^2 grids (measured: 9e-15,
    5e-15 for the linear law, 4e-13 on 16^2).  The complex forward
    model is a complex-safe restatement of the step residual and the outflux
    (branches taken on the real part), itself checked equal to the oracle's on real
    inputs; each complex step is solved by the modified-Picard iteration with the
    operator A taken at the real part, which only drives the iteration (its fixed
    point is R(p) = 0 whatever matrix is used).
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, constitutive, fv, kl, picard

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


# ---------------------------------------------------------------- complex step
def _closure_c(prob, p, Ks):
    """(K, theta) of the Gardner or linear law for complex p (branch on Re p)."""
    if prob["model"] == "gardner":
        unsat = p.real < 0.0
        se = np.where(unsat, np.exp(prob["gardner_a"] * np.where(unsat, p, 0.0)), 1.0)
        return Ks * se, prob["theta_r"] + (prob["theta_s"] - prob["theta_r"]) * se
    return Ks * np.ones_like(p), prob["theta_r"] + prob["c0"] * p


def _residual_c(prob, Ks, p, theta_old):
    """Backward-Euler step residual (net inflow of the harmonic-mean faces minus the
    storage term, Section 4.1) for complex p and Ks, as an n x n array."""
    n = p.shape[0]
    h = 1.0 / n
    K, theta = _closure_c(prob, p, Ks)

    def hm(a, b):
        return 2.0 * a * b / (a + b)
    q = np.zeros_like(p)
    fx = hm(K[:, :-1], K[:, 1:]) * (p[:, :-1] - p[:, 1:]) / h
    q[:, 1:] += fx
    q[:, :-1] -= fx
    fz = hm(K[:-1, :], K[1:, :]) * ((p[:-1, :] - p[1:, :]) / h - 1.0)
    q[1:, :] += fz
    q[:-1, :] -= fz
    q[0, :] += K[0, :] * ((prob["h_bottom"] - p[0, :]) / (0.5 * h) - 1.0)
    q[n - 1, :] += K[n - 1, :] * ((prob["h_top"] - p[n - 1, :]) / (0.5 * h) + 1.0)
    return q / h - (theta - theta_old) / prob["dt"]


def _outflux_c(prob, Ks, p):
    n = p.shape[0]
    h = 1.0 / n
    K, _ = _closure_c(prob, p, Ks)
    return h * np.sum(K[0, :] * ((p[0, :] - prob["h_bottom"]) / (0.5 * h) + 1.0))


def _q_complex(prob, B, xi, n):
    """Q = sum_n dt F(p^n) with every step solved to R = 0 in complex arithmetic."""
    Ks = np.exp(xi @ B).reshape(n, n)  # lognormal marginal (0, 0, 1)
    p = picard.initial_head(prob, n).astype(complex)
    _, theta = _closure_c(prob, p, Ks)
    Q = 0.0
    for _ in range(prob["n_steps"]):
        for it in range(500):
            K, _, C = constitutive.evaluate(prob, p.real, {"Ks": Ks.real})
            kx, kz = fv.face_conductivities(K)
            A = fv.assemble(fv.stencil(kx, kz, C / prob["dt"], 1.0 / n)).toarray()
            r = _residual_c(prob, Ks, p, theta).ravel()
            dp = np.linalg.solve(A, r).reshape(n, n)
            p = p + dp
            if (np.max(np.abs(dp.real)) <= 1e-13 * max(1.0, np.max(np.abs(p.real)))
                    and np.max(np.abs(dp.imag)) <= 1e-13 * max(1e-300, np.max(np.abs(p.imag)))):
                break
        else:
            raise AssertionError("complex step did not converge")
        _, theta = _closure_c(prob, p, Ks)
        Q = Q + prob["dt"] * _outflux_c(prob, Ks, p)
    return Q


def test_complex_restatement_matches_oracle_on_real_inputs():
    prob = _prob()
    _, _, Ks = _fields()
    p = -1.0 - 3.0 * W.uniform_array([11], (N_GRID, N_GRID))
    p[2, 5] = 0.3
    _, th_old, _ = constitutive.evaluate(prob, p - 0.1, {"Ks": Ks})
    r_ref = adjoint.residual(prob, {"Ks": Ks}, p, th_old)
    r_c = _residual_c(prob, Ks.astype(complex), p.astype(complex), th_old).ravel()
    assert np.max(np.abs(r_c.imag)) == 0.0
    assert np.max(np.abs(r_c.real - r_ref)) <= 1e-13 * np.max(np.abs(r_ref))
    f_ref = adjoint.outflux(prob, {"Ks": Ks}, p)
    assert abs(_outflux_c(prob, Ks.astype(complex), p.astype(complex)).real - f_ref) <= 1e-14 * abs(f_ref)


@pytest.mark.parametrize("model,n", [("gardner", 8), ("linear", 8), ("gardner", 16)])
def test_gradient_matches_complex_step(model, n):
    prob = _prob(model, n_steps=3)
    B, xi, Ks = _fields(n=n)
    opts = dict(W.SOLVER, eps_picard=1e-13, max_picard=300)
    r = adjoint.solve_with_gradient(prob, Ks, n, opts, basis=B, marginal=(0.0, 0.0, 1.0), mode="direct")
    assert r["status"] == 0
    t = 1e-30
    for j in range(B.shape[0]):
        x = xi.astype(complex)
        x[j] += 1j * t
        cs = _q_complex(prob, B, x, n).imag / t
        g = r["dQ_dxi"][j]
        assert abs(cs - g) <= 1e-11 * max(abs(cs), 1e-6 * np.max(np.abs(r["dQ_dxi"]))), (j, cs, g)
