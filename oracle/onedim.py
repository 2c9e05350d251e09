"""Independent 1-D column solver (oracle cross-check, FP64).

For fields constant in x the 2-D problem with no-flux sides has an
x-independent solution, which must equal the 1-D cell-centred finite-volume
solution of the same column problem.  This module writes the 1-D scheme out on
its own (tridiagonal modified Picard with a banded direct solve), so that an
index or orientation mistake in the 2-D code shows up as a mismatch.

Same discretisation readings as the 2-D oracle: z up, n cells of width h,
harmonic-mean interior faces, Dirichlet faces at distance h/2 with the adjacent
cell's conductivity, gravity in flux form.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import constitutive


def solve_column(problem, fields_col, n, eps=1e-13, max_picard=200, counts=False):
    """Backward Euler + modified Picard (Section 4.1) on a column; returns p at the final time [n]
    (with counts=True also the Picard iterations of every step, the one that met the stopping
    test included)."""
    h, dt = 1.0 / n, problem["dt"]
    gb, gt = problem["h_bottom"], problem["h_top"]
    p = np.full(n, float(problem["h_init"]))
    _, th_old, _ = constitutive.evaluate(problem, p, fields_col)
    its = []
    for _ in range(problem["n_steps"]):
        for _k in range(max_picard):
            K, th, C = constitutive.evaluate(problem, p, fields_col)
            kf = np.empty(n + 1)
            kf[0], kf[n] = K[0], K[-1]
            kf[1:n] = 2.0 * K[:-1] * K[1:] / (K[:-1] + K[1:])
            dist = np.full(n + 1, h)
            dist[0] = dist[n] = 0.5 * h
            # upward flux through face m (between cells m-1 and m): kf ((p_{m-1} - p_m)/d - 1)
            pl = np.concatenate([[gb], p])
            pr = np.concatenate([p, [gt]])
            flux = kf * ((pl - pr) / dist - 1.0)
            inflow = (flux[:-1] - flux[1:]) / h
            f = inflow - (th - th_old) / dt
            coef = kf / (dist * h)
            diag = coef[:-1] + coef[1:] + C / dt
            ab = np.zeros((3, n))
            ab[0, 1:] = -coef[1:n]
            ab[1, :] = diag
            ab[2, :-1] = -coef[1:n]
            dp = sla.solve_banded((1, 1), ab, f)
            p = p + dp
            if np.max(np.abs(dp)) < eps:
                break
        its.append(_k + 1)
        _, th_old, _ = constitutive.evaluate(problem, p, fields_col)
    return (p, its) if counts else p
