"""Closure laws theta(p), C(p) = d theta/dp and K(p) = Ks * K_rw(p) (oracle, FP64).

van Genuchten-Mualem: Section 2.1, eqs. Sw (saturation), sc_van (moisture
capacity) and Krw (Mualem relative conductivity, closed form of eq. Krw1).
Gardner (exponential) law: the closure used by the benchmark workloads; its
saturated branch (p >= 0) mirrors the vG convention of eq. Sw: S = 1, C = 0,
K_rw = 1.
Linear law (test only): K independent of p and theta affine in p, for which one
modified-Picard step with an exact linear solve is exact.

Every function takes NumPy arrays (or scalars) and returns (K, theta, C).
"""
from __future__ import annotations

import numpy as np


def gardner(p, Ks, a, theta_r, theta_s):
    """Gardner law: S_e = exp(a p) for p < 0, else 1; K = Ks S_e; C = (theta_s-theta_r) a S_e (p < 0)."""
    p = np.asarray(p, dtype=np.float64)
    unsat = p < 0.0
    se = np.where(unsat, np.exp(a * np.minimum(p, 0.0)), 1.0)
    K = Ks * se
    theta = theta_r + (theta_s - theta_r) * se
    C = np.where(unsat, (theta_s - theta_r) * a * se, 0.0)
    return K, theta, C


def vg_saturation(p, alpha, n):
    """Effective saturation S_w(p) of eq. Sw: (1 + |alpha p|^n)^(-m), m = 1 - 1/n, for p < 0; 1 otherwise."""
    p = np.asarray(p, dtype=np.float64)
    m = 1.0 - 1.0 / n
    u = np.abs(alpha * np.minimum(p, 0.0)) ** n
    return np.where(p < 0.0, (1.0 + u) ** (-m), 1.0)


def van_genuchten(p, Ks, alpha, n, theta_r, theta_s):
    """van Genuchten-Mualem law, eqs. Sw, sc_van and Krw.

    In eq. Krw the factor 1 - S^(1/m) is evaluated through the exact identity
    1 - S^(1/m) = |alpha p|^n / (1 + |alpha p|^n), which follows from eq. Sw and
    avoids cancellation as p -> 0- (where the paper notes K_rw is not Lipschitz).
    """
    p = np.asarray(p, dtype=np.float64)
    m = 1.0 - 1.0 / n
    unsat = p < 0.0
    ap = np.abs(alpha * np.minimum(p, 0.0))
    u = ap ** n
    S = (1.0 + u) ** (-m)
    one_minus_S1m = u / (1.0 + u)
    krw = np.sqrt(S) * (1.0 - one_minus_S1m ** m) ** 2
    K = Ks * np.where(unsat, krw, 1.0)
    theta = theta_r + (theta_s - theta_r) * np.where(unsat, S, 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        C_unsat = (theta_s - theta_r) * alpha * m * n * (1.0 + u) ** (-(m + 1.0)) * ap ** (n - 1.0)
    C = np.where(unsat, C_unsat, 0.0)
    return K, theta, C


def linear(p, Ks, c0, theta_r):
    """Test-only linear law: K = Ks, theta = theta_r + c0 p, C = c0."""
    p = np.asarray(p, dtype=np.float64)
    K = Ks * np.ones_like(p)
    theta = theta_r + c0 * p
    C = c0 * np.ones_like(p)
    return K, theta, C


def evaluate(problem: dict, p, fields: dict):
    """Dispatch on problem['model'] with per-cell field arrays (Ks, and alpha, n for vG)."""
    model = problem["model"]
    if model == "gardner":
        return gardner(p, fields["Ks"], problem["gardner_a"], problem["theta_r"], problem["theta_s"])
    if model == "vg":
        return van_genuchten(p, fields["Ks"], fields["alpha"], fields["n"],
                             problem["theta_r"], problem["theta_s"])
    if model == "linear":
        return linear(p, fields["Ks"], problem["c0"], problem["theta_r"])
    raise ValueError(f"unknown closure model {model!r}")


def effective_saturation(problem: dict, p, fields: dict):
    """S_e = (theta - theta_r) / (theta_s - theta_r) (the quantity averaged by the mean-saturation QoI)."""
    _, theta, _ = evaluate(problem, p, fields)
    return (theta - problem["theta_r"]) / (problem["theta_s"] - problem["theta_r"])
