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

Sign convention: each eigenvector is flipped so that its entry of largest
magnitude on the quadrature points is positive.  Degenerate eigenvalues (the
isotropic kernel on a square has mode pairs (a, b) and (b, a)) leave the basis
inside each eigenspace to the eigensolver; quantities invariant under that
choice (eigenvalues, the covariance B^T B of the truncated field) are what may
be compared between independent eigensolvers.
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
    big = np.argmax(np.abs(V), axis=0)
    sign = np.sign(V[big, np.arange(V.shape[1])])
    sign[sign == 0] = 1.0
    V = V * sign
    return lam, V / sw[:, None]


def interpolate(cov, points_q, weights, lam, psi_q, points):
    """Nystrom interpolation Psi_j(x) = (1/lambda_j) sum_q w_q C(x, x_q) Psi_j(x_q); returns [len(points)][M]."""
    out = np.empty((points.shape[0], psi_q.shape[1]))
    for a in range(0, points.shape[0], 2048):
        b = min(a + 2048, points.shape[0])
        out[a:b] = (cov(points[a:b], points_q) * weights[None, :]) @ psi_q / lam[None, :]
    return out


def basis(sigma2, corr_len, n_modes, grids, ref_n=64):
    """KL basis tables B_n[j, c] = sqrt(lambda_j) Psi_j(x_c) for each grid size n (dict n -> [M][n*n])."""
    cov = exponential_cov(sigma2, corr_len)
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
