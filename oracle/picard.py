"""Backward Euler with modified Picard iteration on the mixed form (oracle, FP64).

Section 4.1: on the uniform time grid t^j = j dt, each step solves the mixed
form implicitly (eq. Mixed_based).  Iteration k linearises theta about p^k
(eq. taylorThetap) and solves the correction equation (eq. Mixed_based_3)

    (C^k/dt) dp - div(K^k grad dp) = f~(p^k),    p^{k+1} = p^k + dp,

stopping when ||dp||_inf < eps_PI.  The paper gives up on a sample after 50
Picard iterations (Section 4.3); the limit is a parameter here.

Two ways of solving each correction equation:
  * mode "direct": sparse LU of the assembled five-point matrix (scipy spsolve);
    run to a tight eps_PI this reaches the discrete fixed point R(p) = 0
    independently of any multigrid detail ("fixed-point oracle");
  * mode "mg": multigrid cycles of ``mg.cycle`` (one cycle per Picard step, or,
    with cycles_per_picard = 0, cycles until ||L dp - f~||_inf < eps_MG as in
    Section 4.2) - the same iteration the GPU path runs ("twin oracle").
Readings: p^{j+1,0} = p^j; dp starts from zero; the first iterate of a step
counts as Picard iteration 1.

Fallback (a reading for the benchmark workloads, not in the paper): with
opts["fallback_cycles"] > 0 a sample whose first attempt fails (iteration limit or a
non-finite correction) is integrated again from its initial state with that many
cycles per Picard step and opts["fallback_max_picard"] iterations per step; the
iteration counts of both attempts are reported.  Reason: with one V-cycle per
Picard step the modified Picard iteration stalls or oscillates on some draws of the
Gardner workload where two cycles per step converge (on some of them exact linear
solves stall as well), and dropping such samples would bias the level estimates.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import constitutive, fv, mg

STATUS_OK, STATUS_MAXITER, STATUS_NONFINITE = 0, 1, 2


def _linear_solve(kx, kz, cdt, f, opts, mode, stats):
    n = f.shape[0]
    if mode == "direct":
        A = fv.assemble(fv.stencil(kx, kz, cdt, 1.0 / n))
        stats["cycles"] += 1
        return spla.spsolve(A.tocsc(), f.ravel()).reshape(f.shape)
    levels = mg.hierarchy(kx, kz, cdt, opts.get("coarsest_n", 4))
    gamma = 2 if opts.get("cycle", "V") == "W" else 1
    nu1, nu2 = opts.get("nu1", 2), opts.get("nu2", 2)
    smoother = opts.get("smoother", "rb")
    ncyc = opts.get("cycles_per_picard", 1)
    u = np.zeros_like(f)
    if ncyc > 0:
        for _ in range(ncyc):
            u = mg.cycle(levels, f, u, 0, gamma, nu1, nu2, smoother)
            stats["cycles"] += 1
        return u
    eps_mg = opts.get("eps_mg", 1e-5)
    for _ in range(opts.get("max_cycles", 200)):
        u = mg.cycle(levels, f, u, 0, gamma, nu1, nu2, smoother)
        stats["cycles"] += 1
        if np.max(np.abs(fv.apply_stencil(levels[0].st, u) - f)) < eps_mg:
            break
    return u


def picard_step(problem, fields, p_old, theta_old, opts, mode, stats):
    """One implicit time step; returns (p_new, theta_new, status, picard iterations, last ||dp||)."""
    n = p_old.shape[0]
    h, dt = 1.0 / n, problem["dt"]
    gb, gt = problem["h_bottom"], problem["h_top"]
    p = p_old.copy()
    eps, kmax = opts.get("eps_picard", 1e-8), opts.get("max_picard", 100)
    dpn = np.inf
    for k in range(1, kmax + 1):
        K, theta, C = constitutive.evaluate(problem, p, fields)
        kx, kz = fv.face_conductivities(K)
        f = fv.picard_rhs(p, theta, theta_old, kx, kz, h, dt, gb, gt)
        if not (np.all(np.isfinite(f)) and np.all(np.isfinite(kz)) and np.all(np.isfinite(C))):
            # a blown-up iterate: this iteration's correction cannot be finite
            stats["cycles"] += 1 if mode == "direct" else max(1, opts.get("cycles_per_picard", 1))
            return p, theta, STATUS_NONFINITE, k, float("nan")
        dp = _linear_solve(kx, kz, C / dt, f, opts, mode, stats)
        p = p + dp
        dpn = float(np.max(np.abs(dp)))
        if not np.isfinite(dpn) or not np.all(np.isfinite(p)):
            return p, theta, STATUS_NONFINITE, k, dpn
        if dpn < eps:
            _, theta_new, _ = constitutive.evaluate(problem, p, fields)
            return p, theta_new, STATUS_OK, k, dpn
    _, theta_new, _ = constitutive.evaluate(problem, p, fields)
    return p, theta_new, STATUS_MAXITER, kmax, dpn


def bottom_outflux(problem, fields, p):
    """Downward flux through the bottom Dirichlet face, h * sum_i K_i0 ((p_i0 - g_B)/(h/2) + 1)."""
    n = p.shape[0]
    h = 1.0 / n
    K, _, _ = constitutive.evaluate(problem, p, fields)
    return h * float(np.sum(K[0, :] * ((p[0, :] - problem["h_bottom"]) / (0.5 * h) + 1.0)))


def initial_head(problem, n):
    """Initial pressure head: uniform h_init, or, when the problem gives init_rate, the
    infiltration problem's profile h_init (1 - exp(-init_rate z)) at the cell centres
    (Section 4.3, eq. travellingwave, with h_init = -0.4 and init_rate = 80)."""
    rate = problem.get("init_rate")
    if not rate:
        return np.full((n, n), float(problem["h_init"]))
    z = (np.arange(n) + 0.5) / n
    return np.repeat((problem["h_init"] * (1.0 - np.exp(-rate * z)))[:, None], n, axis=1)


def solve(problem, fields, n, opts, mode="mg", p0=None, record=False):
    """Integrate one sample over problem['n_steps'] steps (with the fallback attempt of the
    module docstring when opts asks for one).

    fields: dict of n x n arrays (Ks, and alpha/n for van Genuchten).
    Returns dict(p, status, picard (per-step counts of every attempt), cycles, dp_last,
    outflux, history, attempts).
    """
    if not all(np.all(np.isfinite(v)) for v in fields.values()):
        # input validation: fields with a non-finite value are not solved
        p = initial_head(problem, n) if p0 is None else np.array(p0, dtype=np.float64)
        return dict(p=p, status=STATUS_NONFINITE, picard=[], cycles=0, dp_last=float("nan"), outflux=0.0,
                    history=[], attempts=1)
    r = _integrate(problem, fields, n, opts, mode, p0, record)
    r["attempts"] = 1
    fb = opts.get("fallback_cycles", 0)
    if r["status"] == STATUS_OK or not fb or mode != "mg":
        return r
    second = _integrate(problem, fields, n, dict(opts, cycles_per_picard=fb, max_picard=opts["fallback_max_picard"]),
                        mode, p0, record)
    second["picard"] = r["picard"] + second["picard"]
    second["cycles"] += r["cycles"]
    second["attempts"] = 2
    return second


def _integrate(problem, fields, n, opts, mode, p0, record):
    """One attempt: backward-Euler steps from the initial state with the given solver options."""
    p = initial_head(problem, n) if p0 is None else np.array(p0, dtype=np.float64)
    _, theta, _ = constitutive.evaluate(problem, p, fields)
    stats = {"cycles": 0}
    counts, hist = [], []
    status, dpn = STATUS_OK, 0.0
    outflux = 0.0
    for _ in range(problem["n_steps"]):
        p, theta, status, k, dpn = picard_step(problem, fields, p, theta, opts, mode, stats)
        counts.append(k)
        if record:
            hist.append(p.copy())
        if status != STATUS_OK:
            break
        outflux += problem["dt"] * bottom_outflux(problem, fields, p)
    return dict(p=p, status=status, picard=counts, cycles=stats["cycles"], dp_last=dpn,
                outflux=outflux, history=hist)
