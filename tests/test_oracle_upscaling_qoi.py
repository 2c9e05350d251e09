"""Pins for three oracle functions that the other tests leave loose.

  * ``mg.coarsen`` on a heterogeneous hierarchy (Section 4.2, coefficient-upscaling
    figure): fine faces carry harmonic means of cell values, every coarser face the
    arithmetic mean of the two finer faces it spans, and a coarse Dirichlet face
    enters the centre coefficient as 2 K / H^2.  With constant K harmonic and
    arithmetic means coincide, so only distinct face values can tell them apart; the
    expected numbers below are worked out by hand from the figure's description.
  * ``qoi.mean_saturation``: the unweighted cell mean of the effective saturation
    (theta - theta_r) / (theta_s - theta_r) at the final time.
  * ``picard.bottom_outflux``: the downward flux through the bottom Dirichlet face,
    h sum_i K_i0 ((p_i0 - g_B) / (h/2) + 1) (gravity along -z, Darcy's law q = -K (grad p + e_z)).

Each test's docstring names the plausible mistakes it rejects.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import constitutive, fv, kl, mg, picard, qoi

# ----------------------------------------------------------------- upscaling


def _fine_faces_4x4():
    """Distinct face values on a 4 x 4 grid.  kx[j, i]: x-face left of cell i in row j
    (columns 0 and 4 are the no-flux sides); kz[j, i]: z-face below row j (rows 0 and 4
    are the bottom and top Dirichlet faces)."""
    kx = np.array([[0.0, 2.0, 4.0, 6.0, 0.0],
                   [0.0, 10.0, 12.0, 14.0, 0.0],
                   [0.0, 20.0, 22.0, 24.0, 0.0],
                   [0.0, 40.0, 42.0, 44.0, 0.0]])
    kz = np.array([[1.0, 3.0, 5.0, 7.0],
                   [2.0, 6.0, 10.0, 14.0],
                   [20.0, 30.0, 40.0, 50.0],
                   [8.0, 16.0, 24.0, 32.0],
                   [9.0, 11.0, 13.0, 15.0]])
    cdt = np.arange(1.0, 17.0).reshape(4, 4)
    return kx, kz, cdt


def test_coarsen_hand_worked_4x4():
    """4 x 4 -> 2 x 2 by hand:
      x-faces: coarse face I of coarse row J spans fine faces 2I of rows 2J and 2J+1,
        kxc[0,1] = (4 + 12)/2 = 8, kxc[1,1] = (22 + 42)/2 = 32, the sides stay 0;
      z-faces: coarse face J of column I spans fine faces 2J of columns 2I and 2I+1,
        bottom (2 + ... ) kzc[0] = ((1+3)/2, (5+7)/2) = (2, 6), interior kzc[1] = (25, 45),
        top kzc[2] = ((9+11)/2, (13+15)/2) = (10, 14);
      C/dt: mean of the four fine cells = [[3.5, 5.5], [11.5, 13.5]].
    Rejects: averaging the wrong pair of fine faces (swapped axis: kxc[0,1] would be
    (4+6)/2 = 5, kzc[1,0] (20+8)/2 = 14), a harmonic mean at the coarse level
    (HM(4, 12) = 6), a sum instead of a mean, and C/dt not averaged over all four cells."""
    kx, kz, cdt = _fine_faces_4x4()
    c = mg.coarsen(mg.Level(kx, kz, cdt))
    assert c.n == 2
    np.testing.assert_array_equal(c.kx, [[0.0, 8.0, 0.0], [0.0, 32.0, 0.0]])
    np.testing.assert_array_equal(c.kz, [[2.0, 6.0], [25.0, 45.0], [10.0, 14.0]])
    np.testing.assert_array_equal(c.cdt, [[3.5, 5.5], [11.5, 13.5]])


def test_coarse_stencil_hand_worked_4x4():
    """The 2 x 2 coarse stencil (H = 1/2, 1/H^2 = 4) assembled from the upscaled faces:
      cell (J=0, I=0): w = 0 (no-flux side), e = -8*4 = -32, s = 0 (bottom Dirichlet, no
        neighbour), n = -25*4 = -100, centre = 32 + 100 + 3.5 + 2*2*4 = 151.5, where the
        last term is the coarse Dirichlet face 2 Kbar / H^2 with Kbar = (1 + 3)/2;
      cell (J=1, I=1): w = -32*4 = -128, e = 0, s = -45*4 = -180, n = 0 (top Dirichlet),
        centre = 128 + 180 + 13.5 + 2*14*4 = 433.5.
    Rejects: the Dirichlet face entered as Kbar/H^2 or 2 Kbar/h^2 (fine mesh width),
    a dropped C/dt, and a wrong-sign neighbour coefficient."""
    kx, kz, cdt = _fine_faces_4x4()
    c = mg.coarsen(mg.Level(kx, kz, cdt))
    w, e, s, n_, cc = c.st
    assert (w[0, 0], e[0, 0], s[0, 0], n_[0, 0], cc[0, 0]) == (0.0, -32.0, 0.0, -100.0, 151.5)
    assert (w[1, 1], e[1, 1], s[1, 1], n_[1, 1], cc[1, 1]) == (-128.0, 0.0, -180.0, 0.0, 433.5)
    # the remaining two cells
    assert (w[0, 1], e[0, 1], s[0, 1], n_[0, 1]) == (-32.0, 0.0, 0.0, -180.0)
    assert cc[0, 1] == 32.0 + 180.0 + 5.5 + 2 * 6.0 * 4
    assert (w[1, 0], e[1, 0], s[1, 0], n_[1, 0]) == (0.0, -128.0, -100.0, 0.0)
    assert cc[1, 0] == 128.0 + 100.0 + 11.5 + 2 * 10.0 * 4


def test_fine_faces_are_harmonic_means_hand_worked():
    """Level 0 faces from cell conductivities (eq. five_stencil): K = [[1, 3], [2, 6]] on a
    2 x 2 grid gives the x-faces HM(1,3) = 1.5 and HM(2,6) = 3, the interior z-faces
    HM(1,2) = 4/3 and HM(3,6) = 4, and Dirichlet faces equal to the adjacent cell value.
    Rejects an arithmetic mean at the fine level (2 and 4) and a missing factor 2 (0.75)."""
    K = np.array([[1.0, 3.0], [2.0, 6.0]])
    kx, kz = fv.face_conductivities(K)
    np.testing.assert_allclose(kx, [[0.0, 1.5, 0.0], [0.0, 3.0, 0.0]], rtol=1e-15, atol=0)
    np.testing.assert_allclose(kz, [[1.0, 3.0], [4.0 / 3.0, 4.0], [2.0, 6.0]], rtol=1e-15, atol=0)


def test_three_level_hierarchy_averages_arithmetic_means():
    """8 x 8 -> 4 x 4 -> 2 x 2 with x-face values 2^j in fine row j (interior faces only):
    the 2h faces are (2^(2J) + 2^(2J+1))/2 = 1.5, 6, 24, 96 per coarse row, and the 4h faces
    the arithmetic mean of two 2h faces, (1.5 + 6)/2 = 3.75 and (24 + 96)/2 = 60 (the mean of
    the four fine rows they span).  z-faces 3^i in fine column i: 2h faces (3^(2I) +
    3^(2I+1))/2 = 2, 18, 162, 1458, 4h faces (2 + 18)/2 = 10 and (162 + 1458)/2 = 810.
    Rejects harmonic means at any coarse level (HM(1.5, 6) = 2.4) and the averaging of
    faces that do not lie on the coarse face's line."""
    n = 8
    kx = np.zeros((n, n + 1))
    kx[:, 1:n] = (2.0 ** np.arange(n))[:, None]
    kz = np.repeat((3.0 ** np.arange(n))[None, :], n + 1, axis=0)
    levels = mg.hierarchy(kx, kz, np.ones((n, n)), coarsest_n=2)
    assert [lv.n for lv in levels] == [8, 4, 2]
    l1, l2 = levels[1], levels[2]
    np.testing.assert_array_equal(l1.kx[:, 1:4], np.repeat(np.array([[1.5], [6.0], [24.0], [96.0]]), 3, axis=1))
    np.testing.assert_array_equal(l1.kx[:, [0, 4]], 0.0)
    np.testing.assert_array_equal(l2.kx, [[0.0, 3.75, 0.0], [0.0, 60.0, 0.0]])
    np.testing.assert_array_equal(l1.kz, np.repeat(np.array([[2.0, 18.0, 162.0, 1458.0]]), 5, axis=0))
    np.testing.assert_array_equal(l2.kz, np.repeat(np.array([[10.0, 810.0]]), 3, axis=0))
    np.testing.assert_array_equal(l2.cdt, 1.0)


# ----------------------------------------------------------- mean saturation
GARDNER = dict(W.GARDNER_INFILTRATION)
VG = dict(model="vg", theta_r=0.05, theta_s=0.5)


@pytest.mark.parametrize("prob,fields", [
    (GARDNER, {"Ks": np.full((4, 4), 0.7)}),
    (VG, {"Ks": np.full((4, 4), 0.7), "alpha": np.full((4, 4), 2.0), "n": np.full((4, 4), 1.6)}),
])
def test_mean_saturation_of_a_saturated_state_is_one(prob, fields):
    """p >= 0 everywhere (zero and positive heads): every cell is saturated, S_e = 1, mean 1.
    Rejects averaging theta instead of S_e (0.5) and summing instead of averaging (16)."""
    p = np.array([[0.0, 0.5, 3.0, 0.0]] * 4)
    assert qoi.mean_saturation(prob, fields, p) == 1.0


@pytest.mark.parametrize("a,h", [(1.0, -1.3), (0.5, -4.0), (2.0, -0.25)])
def test_mean_saturation_of_uniform_gardner_head(a, h):
    """Uniform head h < 0 under the Gardner law: S_e = e^{a h} in every cell, mean e^{a h}.
    Rejects theta in place of S_e (0.05 + 0.45 e^{ah}), e^{h} without the exponent a, and a
    relative conductivity weighting."""
    prob = dict(GARDNER, gardner_a=a)
    fields = {"Ks": W.uniform_array([31, 1], (6, 6), 0.1, 3.0)}
    got = qoi.mean_saturation(prob, fields, np.full((6, 6), h))
    assert got == pytest.approx(math.exp(a * h), rel=1e-15)


def test_mean_saturation_hand_worked_mixed_state():
    """2 x 2 cells with heads 0, -1, -2, 3 (Gardner, a = 1): (1 + e^-1 + e^-2 + 1) / 4;
    van Genuchten with alpha = 2, n = 2 (m = 1/2) at heads -1, -0.5, 0, -2:
    ((1 + 4)^-1/2 + (1 + 1)^-1/2 + 1 + (1 + 16)^-1/2) / 4."""
    p = np.array([[0.0, -1.0], [-2.0, 3.0]])
    got = qoi.mean_saturation(GARDNER, {"Ks": np.ones((2, 2))}, p)
    assert got == pytest.approx((2.0 + math.exp(-1.0) + math.exp(-2.0)) / 4.0, rel=1e-15)
    pv = np.array([[-1.0, -0.5], [0.0, -2.0]])
    fv_ = {"Ks": np.ones((2, 2)), "alpha": np.full((2, 2), 2.0), "n": np.full((2, 2), 2.0)}
    ref = (5 ** -0.5 + 2 ** -0.5 + 1.0 + 17 ** -0.5) / 4.0
    assert qoi.mean_saturation(VG, fv_, pv) == pytest.approx(ref, rel=1e-14)


# -------------------------------------------------------------- bottom outflux
def test_bottom_outflux_vanishes_in_hydrostatic_state():
    """p = c - z with g_B = c: the bottom cell sits h/2 above the face, p_0 - g_B = -h/2, so
    (p_0 - g_B)/(h/2) + 1 = 0 for any K.  Rejects a gravity sign error (-2 K per face), a
    distance of h instead of h/2 (K/2 per face), and a missing gravity term (-K)."""
    n, c = 16, -3.0
    z = (np.arange(n) + 0.5) / n
    p = np.repeat((c - z)[:, None], n, axis=1)
    prob = dict(GARDNER, h_bottom=c)
    fields = {"Ks": W.uniform_array([32], (n, n), 0.2, 5.0)}
    assert abs(picard.bottom_outflux(prob, fields, p)) < 1e-14


def test_bottom_outflux_hand_worked_two_cells():
    """n = 2 (h = 1/2), Gardner a = 1, bottom heads p_00 = -1, p_01 = -0.5, g_B = -2, Ks = 1:
    K = e^-1, e^-0.5; face terms (p - g_B)/(h/2) + 1 = 1/0.25 + 1 = 5 and 1.5/0.25 + 1 = 7;
    F = h (5 e^-1 + 7 e^-0.5) (downward positive).  Rejects an upward sign convention, a
    missing factor h, and K taken from the boundary value g_B instead of the cell."""
    prob = dict(GARDNER, h_bottom=-2.0)
    p = np.array([[-1.0, -0.5], [-7.0, -7.0]])
    got = picard.bottom_outflux(prob, {"Ks": np.ones((2, 2))}, p)
    assert got == pytest.approx(0.5 * (5.0 * math.exp(-1.0) + 7.0 * math.exp(-0.5)), rel=1e-15)


@pytest.mark.parametrize("hb", [-2.0, -10.0])
def test_bottom_outflux_converges_to_steady_gardner_flux(hb):
    """Steady 1-D Gardner column (Ks = 1, a = 1, top head 0): with the Kirchhoff variable
    Phi = e^h, Darcy's law reads q = -(Phi' + Phi) and the steady profile gives the downward
    flux a [Phi_0 + (Phi_1 - Phi_0)/(1 - e^-a)] at every height, 1.50321 for g_B = -2 and
    1.58198 for g_B = -10.  The discrete outflux at the discrete steady state converges to it
    at first order (the half-cell Dirichlet closure).  Rejects a factor 1/2 in the boundary
    gradient and a gravity sign error (both O(1) errors), and h^2 instead of h as the face
    length (a factor n)."""
    a = 1.0
    phi0, phi1 = math.exp(a * hb) / a, math.exp(0.0) / a
    exact = a * (phi0 + (phi1 - phi0) / (1.0 - math.exp(-a)))
    prob = dict(GARDNER, h_bottom=hb, h_init=hb, dt=10.0, n_steps=10)
    errs = []
    for n in (16, 32, 64):
        r = picard.solve(prob, {"Ks": np.ones((n, n))}, n, dict(W.SOLVER, eps_picard=1e-12, max_picard=400),
                         mode="direct")
        assert r["status"] == 0
        errs.append(abs(picard.bottom_outflux(prob, {"Ks": np.ones((n, n))}, r["p"]) - exact))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) >= 0.9, (errs, rates)
    assert errs[-1] < (5e-3 if hb == -2.0 else 8e-2) * exact, errs  # -10: steep bottom layer


def test_mass_balance_with_top_inflow_and_bottom_outflux(kl_basis_small):
    """Per step and in total: stored water = dt (inflow through the top face - outflux
    through the bottom face).  The top inflow is written here from the Dirichlet top face
    (h sum_i K_i,n-1 ((g_T - p_i,n-1)/(h/2) + 1)); the bottom part is the oracle's
    bottom_outflux, and the accumulated outflux QoI of picard.solve is the right-endpoint
    sum of dt F(p^k).  Rejects a sign or factor error in bottom_outflux (the balance is met
    to 1e-11 of the inflow) and a left-endpoint or missing-dt accumulation."""
    n = 16
    lam, B = kl_basis_small
    xi = W.xi_draws(33, 0, [0], 1, B[n].shape[0])[0, 0]
    fields = {"Ks": kl.lognormal(kl.gaussian_field(xi, B[n])).reshape(n, n)}
    prob = dict(GARDNER, n_steps=3)
    h, dt = 1.0 / n, prob["dt"]
    opts = dict(W.SOLVER, eps_picard=1e-13, max_picard=300)
    r = picard.solve(prob, fields, n, opts, mode="direct", record=True)
    assert r["status"] == 0
    p_prev = picard.initial_head(prob, n)
    total_out = 0.0
    for p in r["history"]:
        _, th0, _ = constitutive.evaluate(prob, p_prev, fields)
        K, th1, _ = constitutive.evaluate(prob, p, fields)
        top = h * np.sum(K[n - 1] * ((prob["h_top"] - p[n - 1]) / (0.5 * h) + 1.0))
        out = picard.bottom_outflux(prob, fields, p)
        stored = h * h * np.sum(th1 - th0)
        assert abs(stored - dt * (top - out)) <= 1e-11 * abs(dt * top), (stored, dt * top, dt * out)
        total_out += dt * out
        p_prev = p
    assert r["outflux"] == pytest.approx(total_out, rel=1e-14)
