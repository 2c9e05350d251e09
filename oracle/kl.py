"""Karhunen-Loeve random fields (oracle, FP64).

Section 3: log Ks = Z is a zero-mean Gaussian field (eqs. RandK, GRF) with the
Matern covariance of eq. nonIsotropic; Z is expanded as
Z(x) = sum_j sqrt(lambda_j) Psi_j(x) xi_j (eq. KLexp) with (lambda_j, Psi_j) the
eigenpairs of the Fredholm problem of eq. Fred, truncated at M terms.

The Fredholm problem is discretised by the Nystrom method: a quadrature rule
(points x_q, weights w_q) turns it into the symmetric eigenproblem
W^{1/2} C W^{1/2} v = lambda v with Psi(x_q) = v_q / sqrt(w_q), so that
sum_q w_q Psi_j(x_q) Psi_k(x_q) = delta_jk; the eigenfunctions are then
evaluated anywhere by the Nystrom interpolation
Psi_j(x) = (1/lambda_j) sum_q w_q C(x, x_q) Psi_j(x_q).

Canonical basis: the isotropic kernel on a square has degenerate eigenvalues
(mode pairs (a, b) and (b, a)), inside which an eigensolver may return any
rotation, differently on different machines.  The oracle therefore replaces
each eigenspace (eigenvalues equal to a relative 1e-8) by the Gram-Schmidt
orthonormalisation of the projections of fixed seeded probe vectors onto it
(the projector does not depend on the rotation), and fixes the sign of a simple
eigenvector by its inner product with a probe.  The eigenfunctions are thereby
defined independently of the eigensolver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.special as sps


def matern(r_tilde, nu, sigma2):
    """Matern covariance of eq. nonIsotropic as a function of the scaled distance r~."""
    r_tilde = np.asarray(r_tilde, dtype=np.float64)
    x = 2.0 * np.sqrt(nu) * r_tilde
    with np.errstate(invalid="ignore"):
        val = sigma2 * (2.0 ** (1.0 - nu) / sps.gamma(nu)) * x ** nu * sps.kv(nu, x)
    return np.where(x > 0.0, val, sigma2)


def exponential_cov(sigma2, corr_len):
    """The nu = 1/2 Matern kernel, isotropic: sigma^2 exp(-sqrt(2) r / corr_len)."""
    def cov(X, Y):
        dx = X[:, None, 0] - Y[None, :, 0]
        dz = X[:, None, 1] - Y[None, :, 1]
        return sigma2 * np.exp(-np.sqrt(2.0) * np.sqrt(dx * dx + dz * dz) / corr_len)
    return cov


def separable_exponential_cov_1d(sigma2, b):
    """1-D kernel sigma^2 exp(-|x - y| / b) (analytic eigenpairs known; used as a pin)."""
    def cov(X, Y):
        return sigma2 * np.exp(-np.abs(X[:, None, 0] - Y[None, :, 0]) / b)
    return cov


def cell_centres(n):
    """Centres of the n x n cell-centred grid on the unit square, ordered c = j*n + i (x fastest)."""
    c = (np.arange(n) + 0.5) / n
    zz, xx = np.meshgrid(c, c, indexing="ij")
    return np.stack([xx.ravel(), zz.ravel()], axis=1)


def nystrom(cov, points, weights, n_modes=None):
    """Eigenpairs of the discretised Fredholm operator, largest first.

    Returns (lam [M], psi_q [Q][M]) with psi_q the eigenfunctions at the quadrature points.
    """
    Q = points.shape[0]
    sw = np.sqrt(weights)
    S = sw[:, None] * cov(points, points) * sw[None, :]
    if n_modes is None or n_modes >= Q:
        lam, V = sla.eigh(S)
    else:
        lam, V = sla.eigh(S, subset_by_index=[Q - n_modes, Q - 1])
    order = np.argsort(-lam, kind="stable")
    lam, V = lam[order], V[:, order]
    V = canonical_eigenvectors(lam, V)
    return lam, V / sw[:, None]


def canonical_eigenvectors(lam, V, rtol=1e-8):
    """Rotation- and sign-free eigenvectors: per cluster of equal eigenvalues, orthonormalised
    projections of seeded probe vectors (PCG64 seed 20190321) onto the cluster's span."""
    Q, M = V.shape
    probes = np.random.Generator(np.random.PCG64(20190321)).standard_normal((Q, M))
    out = np.empty_like(V)
    a = 0
    while a < M:
        b = a + 1
        while b < M and abs(lam[b] - lam[a]) <= rtol * abs(lam[a]):
            b += 1
        span = V[:, a:b]
        for k in range(a, b):
            v = span @ (span.T @ probes[:, k])
            for q in range(a, k):
                v = v - out[:, q] * (out[:, q] @ v)
            out[:, k] = v / np.linalg.norm(v)
        a = b
    return out


def interpolate(cov, points_q, weights, lam, psi_q, points):
    """Nystrom interpolation Psi_j(x) = (1/lambda_j) sum_q w_q C(x, x_q) Psi_j(x_q); returns [len(points)][M]."""
    out = np.empty((points.shape[0], psi_q.shape[1]))
    for a in range(0, points.shape[0], 2048):
        b = min(a + 2048, points.shape[0])
        out[a:b] = (cov(points[a:b], points_q) * weights[None, :]) @ psi_q / lam[None, :]
    return out


def matern_cov(nu, lx, lz, sigma2):
    """The anisotropic Matern kernel of eq. nonIsotropic with Phi = (nu, lambda_x, lambda_z, sigma^2)."""
    def cov(X, Y):
        dx = (X[:, None, 0] - Y[None, :, 0]) / lx
        dz = (X[:, None, 1] - Y[None, :, 1]) / lz
        return matern(np.sqrt(dx * dx + dz * dz), nu, sigma2)
    return cov


def basis(sigma2, corr_len, n_modes, grids, ref_n=64, matern_phi=None):
    """KL basis tables B_n[j, c] = sqrt(lambda_j) Psi_j(x_c) for each grid size n (dict n -> [M][n*n]).

    The covariance is the exponential kernel (Matern nu = 1/2, isotropic, sigma2, corr_len),
    or, if matern_phi = (nu, lambda_x, lambda_z, sigma^2) is given, the Matern kernel of
    eq. nonIsotropic (then sigma2 and corr_len are not used)."""
    cov = exponential_cov(sigma2, corr_len) if matern_phi is None else matern_cov(*matern_phi)
    pts = cell_centres(ref_n)
    w = np.full(ref_n * ref_n, 1.0 / (ref_n * ref_n))
    lam, psi_q = nystrom(cov, pts, w, n_modes)
    out = {}
    for n in grids:
        psi = interpolate(cov, pts, w, lam, psi_q, cell_centres(n))
        out[n] = (np.sqrt(lam)[None, :] * psi).T.copy()
    return lam, out


def gaussian_field(xi, B):
    """G = xi @ B: the truncated KL sum of eq. KLexp for each sample (xi [S][M], B [M][N])."""
    return xi @ B


def lognormal(G, log_mean=0.0, scale=1.0, shift=0.0):
    """Marginal transform v = shift + exp(log_mean + scale G) (eq. RandK with Ks_bl = exp(log_mean))."""
    return shift + np.exp(log_mean + scale * G)
