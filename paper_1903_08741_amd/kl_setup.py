"""Host set-up of the Karhunen-Loeve basis tables (run once per workload, FP64).

The paper's KL expansion (Section 3, eq. KLexp) needs the leading eigenpairs
of the covariance operator (eq. Fred).  This set-up step discretises that
operator with the midpoint (Nystrom) rule on a ref x ref cell-centred grid,
takes its leading eigenpairs with LAPACK, and evaluates the eigenfunctions at
the cell centres of every simulation grid by Nystrom interpolation.  The
returned tables B_n[k][c] = sqrt(lambda_k) Psi_k(x_c) are the operand of the
matrix-core product in ``sample_fields``; they are data, built once on the host
before any solve, not a step of the per-sample path.

Covariance: the Matern kernel of eq. nonIsotropic at nu = 1/2 with equal
correlation lengths, sigma^2 exp(-sqrt(2) r / corr_len).

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


def kl_tables(sigma2, corr_len, n_modes, grids, ref=64, chunk=4096):
    """Return (eigenvalues [M], {n: float64 array [M][n*n]}) for the listed grid sizes."""
    xq, zq = _centres(ref)
    Q = xq.size
    w = 1.0 / Q
    A = w * _kernel(xq, zq, xq, zq, sigma2, corr_len)
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
            B[:, a:b] = (_kernel(x[a:b], z[a:b], xq, zq, sigma2, corr_len) @ coef).T
        tables[n] = B * np.sqrt(vals)[:, None]
    return vals, tables
