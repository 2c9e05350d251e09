"""Discrete adjoint of the backward-Euler / modified-Picard solve (oracle, FP64).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

The paper has no adjoint; this is the exact derivative of the discrete forward
model of Sections 4.1-4.2 as the oracle defines it (fv.py, picard.py).  Step n
solves R^n(p^n, p^{n-1}) = 0 with

    R^n(p, p_old) = net_inflow(p; K(p)) - (theta(p) - theta(p_old)) / dt,

K(p) = Ks K_rw(p) per cell and harmonic-mean faces (eq. five_stencil).  The
quantity of interest is the time-integrated downward flux through the bottom
Dirichlet face, Q = sum_{n=1}^{N} dt F(p^n), F(p) = h sum_i K_i0 ((p_i0 - g_B) /
(h/2) + 1).  With the Lagrangian L = Q - sum_n lambda_n^T R^n:

    J_n^T lambda_n = dt dF/dp(p^n) - (dR^{n+1}/dp^n)^T lambda_{n+1},  lambda_{N+1} = 0,
    dR^{n+1}/dp^n = diag(C(p^n)) / dt,
    dQ/dlog Ks = sum_n [dt dF/dlog Ks(p^n) - (dR^n/dlog Ks)^T lambda_n],

J_n = dR^n/dp^n the exact Jacobian: the modified-Picard operator -A (its
C/dt diagonal and face conductivities at p^n) plus the terms of dK/dp.  The
gradient with respect to the KL coefficients follows from Ks = shift +
exp(log_mean + scale G), G = sum_j xi_j B_j (Section 3 eqs. KLexp, RandK).

Every Jacobian is assembled as a sparse matrix and every adjoint system solved
by sparse LU: no iteration, no multigrid.  Models: Gardner and the linear test
law (the closures whose dK/dp is written here).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import constitutive, fv, picard


def dK_dp(problem, p, fields):
    """dK/dp per cell: Gardner a K (p < 0) or 0 (saturated); linear law 0."""
    K, _, _ = constitutive.evaluate(problem, p, fields)
    if problem["model"] == "gardner":
        return np.where(p < 0.0, problem["gardner_a"] * K, 0.0)
    if problem["model"] == "linear":
        return np.zeros_like(p)
    raise ValueError("adjoint oracle: Gardner and linear closures only")


def _face_terms(problem, p):
    """Faces as (cell into which the inflow counts, other cell or -1, t) with the inflow
    K_f * t into the first cell (t of eq. Mixed_based_3's flux per cell area)."""
    n = p.shape[0]
    h = 1.0 / n
    idx = np.arange(n * n).reshape(n, n)
    out = []
    # x-faces: inflow into the right cell b from the left cell a
    a, b = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    out.append((b, a, (p[:, :-1] - p[:, 1:]).ravel() / (h * h)))
    # z-faces: inflow into the upper cell b from the lower cell a (gravity opposes)
    a, b = idx[:-1, :].ravel(), idx[1:, :].ravel()
    out.append((b, a, (((p[:-1, :] - p[1:, :]) / h - 1.0) / h).ravel()))
    # Dirichlet bottom and top faces (face conductivity = the cell's own)
    c = idx[0, :]
    out.append((c, -np.ones_like(c), ((problem["h_bottom"] - p[0, :]) / (0.5 * h) - 1.0) / h))
    c = idx[n - 1, :]
    out.append((c, -np.ones_like(c), ((problem["h_top"] - p[n - 1, :]) / (0.5 * h) + 1.0) / h))
    return out


def flux_derivative(problem, p, K, X):
    """Sparse matrix M with M[r, c] = d(net inflow into r)/dK_c * X_c: the derivative of
    R through the cell conductivities, each column scaled by X_c (X = dK/dp gives the
    dK/dp part of the Jacobian, X = K the derivative in log Ks)."""
    n = p.shape[0]
    Kf = K.ravel()
    Xf = X.ravel()
    rows, cols, vals = [], [], []
    for into, other, t in _face_terms(problem, p):
        inner = other >= 0
        b, a, ti = into[inner], other[inner], t[inner]
        if b.size:
            Ka, Kb = Kf[a], Kf[b]
            s2 = (Ka + Kb) ** 2
            dKa = 2.0 * Kb * Kb / s2   # d hmean / dK_a
            dKb = 2.0 * Ka * Ka / s2
            # inflow into b is K_f t, into a it is -K_f t
            rows += [b, b, a, a]
            cols += [a, b, a, b]
            vals += [ti * dKa * Xf[a], ti * dKb * Xf[b], -ti * dKa * Xf[a], -ti * dKb * Xf[b]]
        c, tc = into[~inner], t[~inner]
        if c.size:
            rows.append(c)
            cols.append(c)
            vals.append(tc * Xf[c])
    N = n * n
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def residual(problem, fields, p, theta_old):
    """R(p, p_old) of one backward-Euler step (theta_old = theta(p_old)), flattened."""
    n = p.shape[0]
    K, theta, _ = constitutive.evaluate(problem, p, fields)
    kx, kz = fv.face_conductivities(K)
    r = fv.picard_rhs(p, theta, theta_old, kx, kz, 1.0 / n, problem["dt"], problem["h_bottom"], problem["h_top"])
    return r.ravel()


def jacobian(problem, fields, p):
    """Exact dR/dp at p: -A (modified-Picard operator) + dK/dp terms."""
    n = p.shape[0]
    K, _, C = constitutive.evaluate(problem, p, fields)
    kx, kz = fv.face_conductivities(K)
    A = fv.assemble(fv.stencil(kx, kz, C / problem["dt"], 1.0 / n))
    return (-A + flux_derivative(problem, p, K, dK_dp(problem, p, fields))).tocsc()


def outflux(problem, fields, p):
    """F(p): downward flux through the bottom Dirichlet face."""
    return picard.bottom_outflux(problem, fields, p)


def outflux_derivatives(problem, fields, p):
    """(dF/dp, dF/dlog Ks), flattened."""
    n = p.shape[0]
    h = 1.0 / n
    K, _, _ = constitutive.evaluate(problem, p, fields)
    Kp = dK_dp(problem, p, fields)
    gp = np.zeros_like(p)
    gk = np.zeros_like(p)
    phi = (p[0, :] - problem["h_bottom"]) / (0.5 * h) + 1.0
    gp[0, :] = h * (Kp[0, :] * phi + K[0, :] / (0.5 * h))
    gk[0, :] = h * K[0, :] * phi
    return gp.ravel(), gk.ravel()


def solve_with_gradient(problem, Ks, n, opts, basis=None, marginal=(0.0, 0.0, 1.0), mode="direct"):
    """Forward solve (picard.solve, every step recorded) and the adjoint.

    Returns dict(status, Q, dQ_dlogKs [n*n], dQ_dxi [M] if basis is given, history, lam).
    """
    fields = {"Ks": Ks}
    r = picard.solve(problem, fields, n, opts, mode=mode, record=True)
    if r["status"] != picard.STATUS_OK:
        return dict(status=r["status"], Q=np.nan, dQ_dlogKs=None, dQ_dxi=None)
    dt = problem["dt"]
    P = r["history"]  # p^1 .. p^N
    N = len(P)
    K_hist = [constitutive.evaluate(problem, q, fields) for q in P]
    lam_next = np.zeros(n * n)
    g = np.zeros(n * n)
    lams = [None] * N
    for k in range(N - 1, -1, -1):
        p = P[k]
        K, _, C = K_hist[k]
        dFp, dFk = outflux_derivatives(problem, fields, p)
        rhs = dt * dFp
        if k < N - 1:
            rhs = rhs - (C.ravel() / dt) * lam_next
        lam = spla.spsolve(jacobian(problem, fields, p).T.tocsc(), rhs)
        E = flux_derivative(problem, p, K, K)
        g += dt * dFk - E.T @ lam
        lams[k] = lam
        lam_next = lam
    out = dict(status=0, Q=r["outflux"], dQ_dlogKs=g, history=P, lam=lams)
    if basis is not None:
        shift, _, scale = marginal
        Kf = Ks.ravel()
        dG = g * scale * (Kf - shift) / Kf
        out["dQ_dxi"] = basis @ dG
    return out
