"""Multilevel Monte Carlo level estimator (oracle, FP64).

Section 5.1: E[P_L] = E[P_0] + sum_l E[P_l - P_{l-1}] (eq. telescope); each term
is a plain MC mean over N_l i.i.d. samples (eqs. MLMCestimator, SMC) where the
fine and coarse members of a pair use the same random input and P_{-1} = 0.
Variances follow eqs. ML_var, MC_var and the level variance eq. level_var.

Sums are taken with math.fsum (correctly rounded), so these are the exact
rounded values of the defining sums.
"""
from __future__ import annotations

import math

import numpy as np


def level_sums(q_fine, q_coarse=None):
    """Sums over the successful pairs of one level.

    q_fine, q_coarse: per-sample QoIs (q_coarse None on level 0, meaning P_{-1} = 0);
    NaN marks a failed sample, and a pair with a failed member is excluded.
    """
    qf = np.asarray(q_fine, dtype=np.float64)
    qc = np.zeros_like(qf) if q_coarse is None else np.asarray(q_coarse, dtype=np.float64)
    ok = np.isfinite(qf) & np.isfinite(qc)
    qf, qc = qf[ok], qc[ok]
    y = qf - qc
    return dict(
        n=int(ok.sum()), n_failed=int((~ok).sum()),
        sY=math.fsum(y), sY2=math.fsum(y * y),
        sQf=math.fsum(qf), sQf2=math.fsum(qf * qf),
        sQc=math.fsum(qc), sQc2=math.fsum(qc * qc),
    )


def mc_mean(s, key="sY"):
    """E^MC_N (eq. SMC) from a sums dict."""
    return s[key] / s["n"]


def mc_var(s, key="Y"):
    """V^MC_N (eq. MC_var): (sum x^2 - (sum x)^2 / N) / (N - 1)."""
    n = s["n"]
    return (s["s" + key + "2"] - s["s" + key] ** 2 / n) / (n - 1)


def combine(level_list):
    """ML estimate of the mean (eq. MLMCestimator) and variance (eq. ML_var), plus per-level V_l."""
    mean = math.fsum(mc_mean(s) for s in level_list)
    var = math.fsum(mc_var(s, "Qf") - (mc_var(s, "Qc") if i > 0 else 0.0)
                    for i, s in enumerate(level_list))
    vl = [mc_var(s, "Y") for s in level_list]
    return dict(mean=mean, var=var, level_var=vl)


def optimal_samples(eps, V, W, integer=True):
    """N_l = eps^-2 (sum_k sqrt(V_k W_k)) sqrt(V_l / W_l) (eq. MLMCSAMP), rounded up unless integer=False."""
    V, W = np.asarray(V, float), np.asarray(W, float)
    tot = math.fsum(np.sqrt(V * W))
    N = tot * np.sqrt(V / W) / eps ** 2
    return np.ceil(N).astype(int) if integer else N
