"""Pins for the oracle's KL sampler (Section 3) and MLMC estimator (Section 5.1).

KL: the nu = 1/2 Matern kernel reduces to the exponential kernel (through the
library Bessel function); the Nystrom eigenproblem satisfies the trace
identity, orthonormality and its own eigen-equation; on the 1-D exponential
kernel the eigenvalues match the analytic transcendental solutions; sample
covariance of the fields matches the truncated-KL covariance.
MLMC: fsum-based sums are correctly rounded (checked with exact rationals);
telescoping identity; optimal sample counts satisfy the variance constraint.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.optimize as so

import workloads as W
from oracle import kl, mlmc, picard, qoi


def test_matern_half_is_exponential():
    r = np.linspace(0.0, 2.0, 41)
    m = kl.matern(r, 0.5, 1.7)
    X = np.stack([r, np.zeros_like(r)], 1)
    e = kl.exponential_cov(1.7, 1.0)(X, np.zeros((1, 2)))[:, 0]
    np.testing.assert_allclose(m, e, rtol=1e-13)


def test_nystrom_trace_orthonormality_residual():
    ref = 16
    cov = kl.exponential_cov(1.0, 0.3)
    pts = kl.cell_centres(ref)
    w = np.full(ref * ref, 1.0 / ref ** 2)
    lam, psi = kl.nystrom(cov, pts, w)
    assert abs(lam.sum() - 1.0) < 1e-12                     # trace = sigma^2 |D|
    G = (psi * w[:, None]).T @ psi
    assert np.max(np.abs(G - np.eye(len(lam)))) < 1e-11     # sum_q w Psi_j Psi_k = delta
    lhs = (cov(pts, pts) * w[None, :]) @ psi[:, :20]
    assert np.max(np.abs(lhs - psi[:, :20] * lam[None, :20])) < 1e-12
    assert np.all(np.diff(lam) <= 1e-15)
    # Nystrom interpolation reproduces the eigenfunctions at the quadrature points
    back = kl.interpolate(cov, pts, w, lam[:20], psi[:, :20], pts)
    assert np.max(np.abs(back - psi[:, :20])) < 1e-10


def _analytic_eigs_1d(b, L, k):
    """Eigenvalues of exp(-|x-y|/b) on an interval of length L = 2a (Ghanem & Spanos, ch. 2)."""
    a, c = L / 2, 1.0 / b
    om = []
    for j in range(k):
        # even: c - w tan(w a) = 0, w a in (j pi, j pi + pi/2)
        f = lambda x: c - x * math.tan(x * a)
        om.append(so.brentq(f, (j * math.pi + 1e-12) / a, (j * math.pi + math.pi / 2 - 1e-12) / a))
        # odd: w + c tan(w a) = 0, w a in (j pi + pi/2, (j+1) pi)
        g = lambda x: x + c * math.tan(x * a)
        om.append(so.brentq(g, (j * math.pi + math.pi / 2 + 1e-12) / a, ((j + 1) * math.pi - 1e-12) / a))
    om = np.sort(np.array(om))
    return 2 * c / (om ** 2 + c ** 2)


def test_nystrom_matches_analytic_1d_eigenvalues():
    """Midpoint Nystrom eigenvalues converge at second order to the analytic ones."""
    b, k = 0.3, 8
    exact = _analytic_eigs_1d(b, 1.0, k)
    lams, errs = [], []
    for m in (200, 400, 800):
        pts = np.stack([(np.arange(m) + 0.5) / m, np.zeros(m)], 1)
        lam, _ = kl.nystrom(kl.separable_exponential_cov_1d(1.0, b), pts, np.full(m, 1.0 / m), 2 * k)
        lams.append(lam[:2 * k])
        errs.append(np.abs(lam[:2 * k] - exact) / exact)
    for e0, e1 in zip(errs[:-1], errs[1:]):
        rates = np.log2(e0 / e1)
        assert np.all((rates > 1.95) & (rates < 2.05)), rates
    assert np.max(errs[-1]) < 3e-4
    richardson = (4 * lams[2] - lams[1]) / 3
    assert np.max(np.abs(richardson - exact) / exact) < 1e-6


def test_field_sample_covariance(kl_basis_small):
    lam, B = kl_basis_small
    n = 8
    Bn = B[n]
    S = 4000
    xi = W.xi_draws(11, 0, range(S), 1, Bn.shape[0])[:, 0, :]
    G = kl.gaussian_field(xi, Bn)
    cov_exact = Bn.T @ Bn
    cov_hat = np.cov(G.T)
    var = np.diag(cov_exact)
    # standard error of a sample covariance ~ sqrt((c_xy^2 + c_xx c_yy)/S)
    se = np.sqrt((cov_exact ** 2 + np.outer(var, var)) / S)
    assert np.max(np.abs(cov_hat - cov_exact) / se) < 5.0
    # truncated pointwise variance cannot exceed sigma^2 and approaches it
    assert np.all(var <= 1.0 + 1e-12) and np.mean(var) > 0.75


def test_lognormal_marginal():
    G = np.array([-1.0, 0.0, 2.0])
    np.testing.assert_allclose(kl.lognormal(G, 0.5, 2.0, 1.0), 1.0 + np.exp(0.5 + 2.0 * G), rtol=1e-15)


def test_level_sums_are_correctly_rounded():
    vals = W.normal_array([12], 1000) * np.exp(W.normal_array([13], 1000) * 10)
    s = mlmc.level_sums(vals)
    exact = sum(Fraction(v) for v in vals)
    assert s["sY"] == float(exact)
    exact2 = sum(Fraction(v) * Fraction(v) for v in vals)
    # the squares are rounded before summation: compare with the sum of rounded squares
    assert s["sY2"] == float(sum(Fraction(float(v * v)) for v in vals))
    assert abs(s["sY2"] - float(exact2)) <= 1e-12 * float(exact2)


def test_failed_pairs_are_excluded():
    s = mlmc.level_sums([1.0, np.nan, 3.0], [0.5, 0.5, np.nan])
    assert s["n"] == 1 and s["n_failed"] == 2 and s["sY"] == 0.5


@pytest.mark.slow
def test_telescoping_identity(kl_basis_small):
    """Equal N_l and the same draws on every level: sum_l mean(Y_l) = mean(Q_L) (eq. telescope)."""
    lam, B = kl_basis_small
    prob = dict(W.GARDNER_INFILTRATION, n_steps=2)
    opts = dict(W.SOLVER)
    grids = (4, 8, 16)
    S = 3
    xi = W.xi_draws(13, 0, range(S), 1, 64)[:, 0, :]
    Q = {}
    for n in grids:
        for s in range(S):
            Ks = kl.lognormal(kl.gaussian_field(xi[s], B[n])).reshape(n, n)
            r = picard.solve(prob, {"Ks": Ks}, n, opts, mode="mg")
            assert r["status"] == 0
            Q[n, s] = qoi.mean_saturation(prob, {"Ks": Ks}, r["p"])
    levels = [mlmc.level_sums([Q[grids[0], s] for s in range(S)])]
    for l in range(1, len(grids)):
        levels.append(mlmc.level_sums([Q[grids[l], s] for s in range(S)],
                                      [Q[grids[l - 1], s] for s in range(S)]))
    est = mlmc.combine(levels)
    direct = math.fsum(Q[grids[-1], s] for s in range(S)) / S
    assert abs(est["mean"] - direct) <= 1e-15 * abs(direct) * 4


def test_optimal_sample_counts_meet_variance_target():
    """eq. MLMCSAMP solves min sum N W s.t. sum V/N = eps^2 (eq. MLMCopt): compare with a numerical optimiser."""
    V = np.array([1e-2, 3e-3, 8e-4, 2e-4])
    Wc = np.array([1.0, 8.0, 64.0, 512.0])
    eps = 1e-2
    N = mlmc.optimal_samples(eps, V, Wc)
    assert np.sum(V / N) <= eps ** 2 * (1 + 1e-12)
    Nr = mlmc.optimal_samples(eps, V, Wc, integer=False)
    assert abs(np.sum(V / Nr) - eps ** 2) <= 1e-12 * eps ** 2
    res = so.minimize(lambda x: np.sum(np.exp(x) * Wc), np.log(Nr) + 0.3, method="SLSQP",
                      constraints=[{"type": "eq", "fun": lambda x: np.sum(V * np.exp(-x)) / eps ** 2 - 1.0}],
                      options={"ftol": 1e-14, "maxiter": 500})
    np.testing.assert_allclose(np.exp(res.x), Nr, rtol=1e-4)


def test_matern_closed_forms():
    """eq. nonIsotropic at nu = 3/2 is (1 + x) e^{-x} with x = 2 sqrt(nu) r~ (the half-integer
    closed form of K_{3/2}); as nu grows it tends to the squared exponential exp(-r~^2)."""
    r = np.linspace(0.0, 3.0, 31)
    x = np.sqrt(6.0) * r
    np.testing.assert_allclose(kl.matern(r, 1.5, 2.0), 2.0 * (1.0 + x) * np.exp(-x), rtol=1e-12, atol=1e-15)
    err = [np.max(np.abs(kl.matern(r, nu, 1.0) - np.exp(-r * r))) for nu in (20.0, 80.0)]
    assert err[1] < 4e-3 and err[1] < err[0] / 3.0  # O(1/nu) approach to the limit


def test_matern_basis_reduces_to_exponential_and_is_anisotropic():
    lam_e, B_e = kl.basis(1.0, 0.3, 12, [8], ref_n=16)
    lam_m, B_m = kl.basis(0.0, 0.0, 12, [8], ref_n=16, matern_phi=(0.5, 0.3, 0.3, 1.0))
    np.testing.assert_allclose(lam_m, lam_e, rtol=1e-12)
    assert np.max(np.abs(B_m[8] - B_e[8])) < 1e-12
    # lambda_z << lambda_x: the field varies faster along z than along x
    lam, B = kl.basis(0.0, 0.0, 40, [16], ref_n=32, matern_phi=(0.5, 0.5, 0.05, 1.0))
    G = (W.normal_array([3], (200, 40)) @ B[16]).reshape(200, 16, 16)
    dz = np.mean(np.diff(G, axis=1) ** 2)
    dx = np.mean(np.diff(G, axis=2) ** 2)
    assert dz > 3.0 * dx
