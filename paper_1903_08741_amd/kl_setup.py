"""Host set-up of the Karhunen-Loeve basis tables (run once per workload, FP64).

The paper's KL expansion (Section 3, eq. KLexp) needs the leading eigenpairs
of the covariance operator (eq. Fred).  This set-up step discretises that
operator with the midpoint (Nystrom) rule on a ref x ref cell-centred grid,
takes its leading eigenpairs with LAPACK, and evaluates the eigenfunctions at
the cell centres of every simulation grid by Nystrom interpolation.  The
returned tables B_n[k][c] = sqrt(lambda_k) Psi_k(x_c) are the operand of the
matrix-core product in ``sample_fields``; they are data, built once on the host
before any solve, not a step of the per-sample path.

Covariance: the Matern kernel of eq. nonIsotropic, by default at nu = 1/2 with
equal correlation lengths, sigma^2 exp(-sqrt(2) r / corr_len); any
Phi = (nu, lambda_x, lambda_z, sigma^2) through ``matern_phi`` (Table Matern:
Phi_1 = (1.0, 0.2, 0.2, 1), Phi_2 = (0.5, 0.1, 0.01, 1)).

The tables must not depend on the eigensolver: inside every eigenspace of
(relatively) equal eigenvalues the basis is rebuilt from the projections of
fixed seeded probe vectors (Gram-Schmidt in probe order), which also fixes the
signs.  Two machines, or the oracle and this set-up, then produce the same
tables up to rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _centres(n):
    t = (np.arange(n, dtype=np.float64) + 0.5) / n
    x = np.tile(t, n)        # i fastest
    z = np.repeat(t, n)
    return x, z


def _kernel(x1, z1, x2, z2, sigma2, corr_len):
    r = np.hypot(x1[:, None] - x2[None, :], z1[:, None] - z2[None, :])
    return sigma2 * np.exp(-np.sqrt(2.0) / corr_len * r)


def _matern_kernel(x1, z1, x2, z2, phi):
    """sigma^2 2^(1-nu)/Gamma(nu) (2 sqrt(nu) r~)^nu K_nu(2 sqrt(nu) r~), r~ scaled per axis."""
    import scipy.special
    nu, lx, lz, sigma2 = phi
    u = 2.0 * np.sqrt(nu) * np.hypot((x1[:, None] - x2[None, :]) / lx, (z1[:, None] - z2[None, :]) / lz)
    out = np.full(u.shape, float(sigma2))
    pos = u > 0.0
    up = u[pos]
    out[pos] = sigma2 * (2.0 ** (1.0 - nu) / scipy.special.gamma(nu)) * up ** nu * scipy.special.kv(nu, up)
    return out


def _fix_eigenspaces(vals, vecs, rtol=1e-8):
    probes = np.random.Generator(np.random.PCG64(20190321)).standard_normal(vecs.shape)
    M = vals.size
    groups, start = [], 0
    for k in range(1, M + 1):
        if k == M or abs(vals[k] - vals[start]) > rtol * abs(vals[start]):
            groups.append((start, k))
            start = k
    fixed = np.zeros_like(vecs)
    for a, b in groups:
        E = vecs[:, a:b]
        P = E @ (E.T @ probes[:, a:b])            # probes projected on the eigenspace
        Qm, Rm = np.linalg.qr(P)                  # Gram-Schmidt in probe order
        fixed[:, a:b] = Qm * np.sign(np.diag(Rm))[None, :]
    return fixed


def kl_tables(sigma2, corr_len, n_modes, grids, ref=64, chunk=4096, matern_phi=None):
    """Return (eigenvalues [M], {n: float64 array [M][n*n]}) for the listed grid sizes.
    With matern_phi = (nu, lambda_x, lambda_z, sigma^2) the covariance is that Matern
    kernel (sigma2 and corr_len are then not used)."""
    if matern_phi is None:
        def kern(a1, b1, a2, b2):
            return _kernel(a1, b1, a2, b2, sigma2, corr_len)
    else:
        def kern(a1, b1, a2, b2):
            return _matern_kernel(a1, b1, a2, b2, matern_phi)
    xq, zq = _centres(ref)
    Q = xq.size
    w = 1.0 / Q
    A = w * kern(xq, zq, xq, zq)
    vals, vecs = scipy.linalg.eigh(A, subset_by_index=[Q - n_modes, Q - 1])
    vals, vecs = vals[::-1].copy(), vecs[:, ::-1].copy()
    vecs = _fix_eigenspaces(vals, vecs)
    psi_q = vecs / np.sqrt(w)                      # sum_q w psi_j psi_k = delta_jk
    coef = psi_q * (w / vals)[None, :]             # Nystrom weights (w / lambda_j) psi_j(x_q)
    tables = {}
    for n in grids:
        x, z = _centres(n)
        B = np.empty((n_modes, n * n))
        for a in range(0, n * n, chunk):
            b = min(a + chunk, n * n)
            B[:, a:b] = (kern(x[a:b], z[a:b], xq, zq) @ coef).T
        tables[n] = B * np.sqrt(vals)[:, None]
    return vals, tables
