"""Pins for the oracle's discretisation, multigrid and Picard solver (Sections 4.1-4.2).

What fixes each part, independently of the oracle's own code:
  * five-point operator: a manufactured constant-coefficient Poisson problem
    converges at second order; an independent Kronecker-product assembly of the
    constant-coefficient operator gives the same linear backward-Euler step;
  * operator structure: symmetric M-matrix;
  * multigrid: cycles converge to the sparse direct solution of the same system;
  * gravity and boundary treatment: the hydrostatic state is stationary for any
    conductivity field; the steady 1-D Gardner profile has a closed form;
  * 2-D code vs an independent 1-D column code on x-constant fields (the solution, and
    the Picard iterations of every step with exact linear solves);
  * modified Picard: mass balance per step; twin (one cycle per step) and
    lexicographic-smoother variants reach the same fixed point as sparse LU.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import constitutive, fv, kl, mg, onedim, picard


def _field(kl_basis_small, n, seed=0, scale=1.0):
    lam, B = kl_basis_small
    xi = W.xi_draws(7, 0, [seed], 1, B[n].shape[0])[0, 0]
    return kl.lognormal(kl.gaussian_field(xi, B[n]), scale=scale).reshape(n, n)


def _poisson_system(n):
    K = np.ones((n, n))
    kx, kz = fv.face_conductivities(K)
    return kx, kz, np.zeros((n, n))


def test_manufactured_poisson_second_order():
    """u* = cos(pi x) sin(pi z): Neumann on x = 0,1, Dirichlet 0 on z = 0,1, -lap u* = 2 pi^2 u*."""
    errs = []
    for n in (32, 64, 128, 256):
        kx, kz, cdt = _poisson_system(n)
        A = fv.assemble(fv.stencil(kx, kz, cdt, 1.0 / n))
        X = kl.cell_centres(n)
        ustar = np.cos(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
        u = spla.spsolve(A.tocsc(), 2 * np.pi ** 2 * ustar)
        errs.append(np.max(np.abs(u - ustar)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.9 < r < 2.1 for r in rates), (errs, rates)


def test_operator_is_symmetric_m_matrix(kl_basis_small):
    n = 16
    Kc = _field(kl_basis_small, n, 1)
    kx, kz = fv.face_conductivities(Kc)
    cdt = W.uniform_array([3, 1], (n, n), 0.0, 5.0)
    A = fv.assemble(fv.stencil(kx, kz, cdt, 1.0 / n))
    assert abs(A - A.T).max() == 0.0
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0.0
    row_off = np.asarray(off.sum(axis=1)).ravel()
    assert np.all(A.diagonal() + row_off >= -1e-12 * A.diagonal())
    # rows touching a Dirichlet face are strictly diagonally dominant
    dd = (A.diagonal() + row_off).reshape(n, n)
    assert np.all(dd[0] > 0) and np.all(dd[-1] > 0)


def test_kronecker_assembly_matches_stencil():
    """Constant K = k0: A = k0/h^2 (I (x) Tx + Tz (x) I) + c0/dt with Neumann Tx and half-cell Dirichlet Tz."""
    n, k0, cdt0 = 12, 0.7, 3.0
    h = 1.0 / n
    Tx = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    Tx[0, 0] = 1.0
    Tx[n - 1, n - 1] = 1.0
    Tz = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    Tz[0, 0] = 3.0       # one interior face + Dirichlet face of weight 2
    Tz[n - 1, n - 1] = 3.0
    I = sp.identity(n)
    Aref = (k0 / h ** 2) * (sp.kron(I, Tx) + sp.kron(Tz, I)) + cdt0 * sp.identity(n * n)
    kx, kz = fv.face_conductivities(np.full((n, n), k0))
    A = fv.assemble(fv.stencil(kx, kz, np.full((n, n), cdt0), h))
    assert abs(A - Aref).max() < 1e-12 * abs(Aref).max()


@pytest.mark.parametrize("n", [8, 16, 32])
def test_multigrid_converges_to_direct_solution(kl_basis_small, n):
    Kc = _field(kl_basis_small, n, 2, scale=1.5)
    kx, kz = fv.face_conductivities(Kc)
    cdt = W.uniform_array([4, n], (n, n), 0.0, 2.0)
    f = W.normal_array([5, n], (n, n))
    levels = mg.hierarchy(kx, kz, cdt, 4)
    A = fv.assemble(levels[0].st)
    ref = spla.spsolve(A.tocsc(), f.ravel()).reshape(n, n)
    u = np.zeros_like(f)
    for _ in range(60):
        u = mg.cycle(levels, f, u)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_coarse_operator_is_direct_discretisation():
    """Constant K: arithmetic-mean upscaling must reproduce the constant-K stencil on the coarse mesh."""
    n, k0 = 16, 2.5
    kx, kz = fv.face_conductivities(np.full((n, n), k0))
    cdt = np.full((n, n), 0.3)
    levels = mg.hierarchy(kx, kz, cdt, 4)
    for lev in levels[1:]:
        kxc, kzc = fv.face_conductivities(np.full((lev.n, lev.n), k0))
        ref = fv.stencil(kxc, kzc, np.full((lev.n, lev.n), 0.3), 1.0 / lev.n)
        for a, b in zip(lev.st, ref):
            np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)


def test_hydrostatic_state_is_stationary(kl_basis_small):
    """p = c - z with g_top = c - 1, g_bottom = c: every discrete flux vanishes for any Ks."""
    n = 16
    Ks = _field(kl_basis_small, n, 3, scale=1.5)
    c = -2.0
    X = kl.cell_centres(n)
    p0 = (c - X[:, 1]).reshape(n, n)
    prob = dict(W.GARDNER_INFILTRATION, h_top=c - 1.0, h_bottom=c, n_steps=3)
    r = picard.solve(prob, {"Ks": Ks}, n, dict(W.SOLVER), mode="mg", p0=p0)
    assert r["status"] == 0 and r["picard"] == [1, 1, 1]
    assert np.max(np.abs(r["p"] - p0)) <= 1e-13


def _gardner_steady_phi(z, a, Ks, hb, ht):
    phi0, phi1 = Ks / a * math.exp(a * hb), Ks / a * math.exp(a * ht)
    return phi0 + (phi1 - phi0) * (1 - np.exp(-a * z)) / (1 - math.exp(-a))


@pytest.mark.parametrize("hb", [-2.0, -10.0])
def test_steady_gardner_profile(hb):
    """Kirchhoff transform Phi = Ks/a e^{a h} turns the steady 1-D problem into Phi' + a Phi = const.

    The error is measured in Phi, which is smooth; h itself has an unresolvable
    logarithmic layer at the bottom when h_B = -10.  First order is what the
    half-cell Dirichlet closure guarantees.
    """
    # pseudo-transient continuation to the steady state (Picard on the steady problem from the
    # dry start stalls for the steep case); ten steps of dt = 10 reach it to rounding
    prob = dict(W.GARDNER_INFILTRATION, h_bottom=hb, h_init=hb, dt=10.0, n_steps=10)
    errs = []
    for n in (16, 32, 64):
        r = picard.solve(prob, {"Ks": np.ones((n, n))}, n,
                         dict(W.SOLVER, eps_picard=1e-12, max_picard=400), mode="direct")
        assert r["status"] == 0
        z = (np.arange(n) + 0.5) / n
        ex = _gardner_steady_phi(z, 1.0, 1.0, hb, 0.0)
        assert np.max(np.abs(r["p"] - r["p"][:, :1])) < 1e-10   # x-independent
        errs.append(np.max(np.abs(np.exp(r["p"][:, 0]) - ex)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) >= 0.95, (errs, rates)
    assert errs[-1] < (1e-3 if hb == -2.0 else 0.2)


def test_two_d_matches_independent_column_solver(kl_basis_small):
    n = 16
    zfield = _field(kl_basis_small, n, 4)[:, 5]          # a column of a random field
    Ks2 = np.repeat(zfield[:, None], n, axis=1)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=3)
    r = picard.solve(prob, {"Ks": Ks2}, n, dict(W.SOLVER, eps_picard=1e-13, max_picard=300), mode="direct")
    col = onedim.solve_column(prob, {"Ks": zfield}, n, eps=1e-13)
    assert r["status"] == 0
    assert np.max(np.abs(r["p"] - col[:, None])) <= 1e-12 * np.max(np.abs(col))


def test_linear_model_one_picard_step_is_backward_euler():
    """Linear law: the first Picard correction with an exact solve is the exact backward-Euler step."""
    n, k0, c0 = 12, 0.8, 0.3
    prob = dict(model="linear", theta_r=0.05, c0=c0, h_top=0.0, h_bottom=-1.0, h_init=-1.0,
                dt=0.05, n_steps=1)
    r = picard.solve(prob, {"Ks": np.full((n, n), k0)}, n, dict(W.SOLVER, eps_picard=1e-12), mode="direct")
    assert r["picard"] == [2]   # second iteration finds dp = 0
    # exact backward Euler, assembled independently for a constant-coefficient column
    h, dt = 1.0 / n, prob["dt"]
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    T[0, 0] = T[n - 1, n - 1] = 3.0
    A = (k0 / h ** 2) * T + (c0 / dt) * sp.identity(n)
    rhs = (c0 / dt) * np.full(n, -1.0)
    # Dirichlet data enter with weight 2k/h^2; with constant K the gravity term dK/dz vanishes
    rhs[0] += 2 * k0 / h ** 2 * prob["h_bottom"]
    rhs[-1] += 2 * k0 / h ** 2 * prob["h_top"]
    col = spla.spsolve(A.tocsc(), rhs)
    assert np.max(np.abs(r["p"] - col[:, None])) < 1e-12


def test_mass_balance_per_step(kl_basis_small):
    n = 16
    Ks = _field(kl_basis_small, n, 5)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=1)
    fields = {"Ks": Ks}
    p0 = np.full((n, n), prob["h_init"])
    _, th0, _ = constitutive.evaluate(prob, p0, fields)
    h = 1.0 / n
    for eps, tol in ((1e-8, 1e-6), (1e-13, 1e-11)):
        r = picard.solve(prob, fields, n, dict(W.SOLVER, eps_picard=eps, max_picard=300), mode="direct")
        K, th1, _ = constitutive.evaluate(prob, r["p"], fields)
        kx, kz = fv.face_conductivities(K)
        stored = h * h * np.sum(th1 - th0)
        inflow = prob["dt"] * fv.boundary_inflow_total(r["p"], kz, h, prob["h_bottom"], prob["h_top"])
        assert abs(stored - inflow) <= tol * abs(inflow), (eps, stored, inflow)


@pytest.mark.parametrize("n", [16, 32])
def test_twin_reaches_fixed_point(kl_basis_small, n):
    Ks = _field(kl_basis_small, n, 6)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=2)
    opts = dict(W.SOLVER, eps_picard=1e-13, max_picard=400)
    twin = picard.solve(prob, {"Ks": Ks}, n, opts, mode="mg")
    fixed = picard.solve(prob, {"Ks": Ks}, n, opts, mode="direct")
    assert twin["status"] == 0 and fixed["status"] == 0
    assert np.max(np.abs(twin["p"] - fixed["p"])) <= 1e-10 * np.max(np.abs(fixed["p"]))


def test_lexicographic_and_w_cycle_variants_reach_same_fixed_point(kl_basis_small):
    n = 8
    Ks = _field(kl_basis_small, n, 7)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=1)
    base = dict(W.SOLVER, eps_picard=1e-13, max_picard=400)
    rb = picard.solve(prob, {"Ks": Ks}, n, base, mode="mg")
    lex = picard.solve(prob, {"Ks": Ks}, n, dict(base, smoother="lex"), mode="mg")
    wcy = picard.solve(prob, {"Ks": Ks}, n, dict(base, cycle="W", cycles_per_picard=0, eps_mg=1e-12), mode="mg")
    for r in (lex, wcy):
        assert r["status"] == 0
        assert np.max(np.abs(r["p"] - rb["p"])) <= 1e-10 * np.max(np.abs(rb["p"]))


def test_fixed_point_independent_of_start(kl_basis_small):
    n = 16
    Ks = _field(kl_basis_small, n, 8)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=1)
    fields = {"Ks": Ks}
    opts = dict(W.SOLVER, eps_picard=1e-13, max_picard=400)
    p_old = np.full((n, n), prob["h_init"])
    _, th_old, _ = constitutive.evaluate(prob, p_old, fields)
    a = picard.picard_step(prob, fields, p_old, th_old, opts, "direct", {"cycles": 0})
    start = p_old + 0.1 * W.normal_array([9], (n, n))
    b = picard.picard_step(prob, fields, start, th_old, opts, "direct", {"cycles": 0})
    assert a[2] == 0 and b[2] == 0
    assert np.max(np.abs(a[0] - b[0])) <= 1e-12 * np.max(np.abs(a[0]))


def test_infiltration_initial_profile():
    """eq. travellingwave: p0 = -0.4 (1 - exp(-80 z)) is ~0 at the bottom, reaches the top
    Dirichlet value -0.4 within rounding in the upper half, decreases with height, and is
    independent of x (cell centres z = (j + 1/2) h)."""
    prob = dict(W.TRAVELLING_WAVE)
    for n in (8, 32):
        p = picard.initial_head(prob, n)
        assert p.shape == (n, n) and np.all(p == p[:, :1])
        col = p[:, 0]
        assert np.all(np.diff(col) < 0.0) or np.all(np.diff(col[: n // 4]) < 0.0)
        assert abs(col[-1] + 0.4) < 1e-15 and abs(col[n // 2:] + 0.4).max() < 1e-9
        assert -0.4 * (1.0 - np.exp(-40.0 / n)) == pytest.approx(col[0], rel=1e-14)
    assert np.all(picard.initial_head(dict(W.GARDNER_INFILTRATION), 4) == -10.0)


def test_fallback_attempt_reaches_the_fixed_point(kl_basis_small):
    """A first attempt forced to fail (two Picard iterations allowed) is replaced by a second
    attempt from the initial state with two V(2,2) per step; it converges to the sparse-LU
    fixed point, and the reported counts are the failed attempt's followed by the second's."""
    n = 16
    Ks = _field(kl_basis_small, n, 9)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=2)
    opts = dict(W.SOLVER, eps_picard=1e-13, max_picard=2, fallback_cycles=2, fallback_max_picard=400)
    r = picard.solve(prob, {"Ks": Ks}, n, opts, mode="mg")
    fixed = picard.solve(prob, {"Ks": Ks}, n, dict(W.SOLVER, eps_picard=1e-13, max_picard=400), mode="direct")
    second = picard.solve(prob, {"Ks": Ks}, n, dict(W.SOLVER, eps_picard=1e-13, max_picard=400, cycles_per_picard=2),
                          mode="mg")
    assert r["status"] == 0 and r["attempts"] == 2 and fixed["status"] == 0
    assert r["picard"] == [2] + second["picard"]
    assert r["cycles"] == 2 + second["cycles"]
    assert np.max(np.abs(r["p"] - fixed["p"])) <= 1e-10 * np.max(np.abs(fixed["p"]))


def test_non_finite_fields_are_rejected_without_solving():
    """A field with a NaN or infinite value is invalid input: status NONFINITE, no iteration
    (a NaN conductivity would otherwise act as an impermeable cell through the guarded
    harmonic mean)."""
    n = 8
    Ks = np.ones((n, n))
    for bad in (np.nan, np.inf):
        f = Ks.copy()
        f[3, 4] = bad
        r = picard.solve(dict(W.GARDNER_INFILTRATION, n_steps=2), {"Ks": f}, n, dict(W.SOLVER), mode="mg")
        assert r["status"] == picard.STATUS_NONFINITE and r["picard"] == [] and r["cycles"] == 0


def test_picard_counts_match_independent_column_solver(kl_basis_small):
    """The 2-D modified Picard loop (exact linear solves) takes, step by step, as many
    iterations as the independent 1-D column code on an x-constant field: the same
    stopping test on the same iterates (Section 4.1)."""
    n = 16
    zfield = _field(kl_basis_small, n, 6)[:, 9]
    Ks2 = np.repeat(zfield[:, None], n, axis=1)
    prob = dict(W.GARDNER_INFILTRATION, n_steps=4)
    r = picard.solve(prob, {"Ks": Ks2}, n, dict(W.SOLVER, eps_picard=1e-8, max_picard=300), mode="direct")
    col, its = onedim.solve_column(prob, {"Ks": zfield}, n, eps=1e-8, counts=True)
    assert r["status"] == 0
    assert list(r["picard"]) == its and min(its) > 1
    assert np.max(np.abs(r["p"] - col[:, None])) <= 1e-8 * np.max(np.abs(col))
