"""Adaptive PC_MLMC (Section 5.1, Algorithm 1): the oracle's loop pinned on
hand-worked cases, and the library's host evaluation of eq. MLMCSAMP against the
oracle's.  No GPU is needed.

Hand-worked cases (W in work units: cycles x cells; a grid (n, 0) pair with one
cycle costs n^2):
  A. one level, Y = 0, 1, 0, 1, ...; N* = 2; eps = 0.3.  Warm-up V = 0.5, so
     N = ceil(0.5 / 0.09) = 6; after six pairs V = (3 - 9/6) / 5 = 0.3 and
     N = ceil(3.33) = 4 <= 6: two updates, six pairs, mean 0.5.
  B. as A, but every third pair fails (i = 2, 5, ...): the six successes take
     eight draws and the failed pairs enter no sum.
  C. two levels, W = (4, 20), Y0 = 0, 2, 0, 2, ..., Y1 = 0, 0.2, ...; N* = (2, 2);
     eps = 0.5.  Warm-up V = (2, 0.02): sum sqrt(VW) = sqrt(8) + sqrt(0.4) =
     3.46088, N = (ceil(9.79), ceil(0.44)) = (10, 2 as the floor of two).  After
     ten level-0 pairs V0 = 10/9 and N = (ceil(5.78), 2): converged after two
     updates with (10, 2) pairs; mean 1.0 + 0.1; variance (eq. ML_var)
     10/9 + 0.02 (coarse member of level 1 constant).
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from oracle import mlmc, pc_mlmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _alt(period_vals):
    return lambda l, i: (period_vals[i % len(period_vals)], None, 1, 0)


def test_case_a_single_level_is_plain_mc():
    drawn = []

    def s(l, i):
        drawn.append(i)
        return (float(i % 2), None, 1, 0)

    r = pc_mlmc.run(s, [(2, 0)], [2], 0.3)
    lv = r["levels"][0]
    assert drawn == list(range(6))
    assert (r["rounds"], lv["drawn"], lv["target"], lv["W"]) == (2, 6, 4, 4.0)
    assert lv["V"] == pytest.approx(0.3, rel=1e-15)
    assert r["mean"] == 0.5 and r["converged"]
    assert r["sampling_err2"] == pytest.approx(0.3 / 6, rel=1e-15)


def test_case_b_failed_pairs_are_replaced():
    def s(l, i):
        return (np.nan if i % 3 == 2 else float(i % 3), None, 1, 0)

    r = pc_mlmc.run(s, [(2, 0)], [2], 0.3)
    lv = r["levels"][0]
    assert lv["drawn"] == 8 and lv["sums"]["n"] == 6 and lv["sums"]["n_failed"] == 2
    assert r["mean"] == 0.5 and r["converged"]


def test_case_c_two_levels_hand_worked():
    def s(l, i):
        if l == 0:
            return (2.0 * (i % 2), None, 1, 0)
        return (1.0 + 0.2 * (i % 2), 1.0, 1, 1)

    r = pc_mlmc.run(s, [(2, 0), (4, 2)], [2, 2], 0.5)
    l0, l1 = r["levels"]
    assert r["rounds"] == 2 and r["converged"]
    assert (l0["drawn"], l1["drawn"]) == (10, 2)
    assert (l0["target"], l1["target"]) == (6, 2)
    assert (l0["W"], l1["W"]) == (4.0, 20.0)
    assert l0["V"] == pytest.approx(10 / 9, rel=1e-15)
    assert r["mean"] == pytest.approx(1.1, rel=1e-15)
    assert r["var"] == pytest.approx(10 / 9 + 0.02, rel=1e-14)


def test_max_rounds_and_max_pairs_stop_unconverged():
    s = _alt([0.0, 1.0])
    r = pc_mlmc.run(s, [(2, 0)], [2], 0.01, max_rounds=1)
    assert r["rounds"] == 1 and not r["converged"]
    r = pc_mlmc.run(s, [(2, 0)], [2], 0.01, max_pairs=20)
    assert r["levels"][0]["drawn"] == 20 and not r["converged"]


def test_final_counts_satisfy_eq_mlmcsamp_and_the_tolerance():
    """On a random three-level sampler, the final targets are eq. MLMCSAMP of the final
    V_l and warm-up W_l, every level holds at least its target, and sum V/N <= eps^2."""
    rng = np.random.default_rng(5)
    sd = [0.3, 0.05, 0.01]
    vals = [rng.standard_normal(100000) * s for s in sd]

    def s(l, i):
        return (1.0 + vals[l][i], 1.0 if l else None, 3 + l, 3 + l if l else 0)

    grids = [(4, 0), (8, 4), (16, 8)]
    r = pc_mlmc.run(s, grids, [10, 10, 10], 0.01)
    V = [x["V"] for x in r["levels"]]
    Wl = [x["W"] for x in r["levels"]]
    assert Wl == [3 * 16.0, 4 * 64.0 + 4 * 16.0, 5 * 256.0 + 5 * 64.0]
    N = mlmc.optimal_samples(0.01, V, Wl)
    for x, n in zip(r["levels"], N):
        assert x["target"] == max(int(n), 2) and x["sums"]["n"] >= x["target"]
    assert r["converged"] and r["sampling_err2"] <= 1e-4
    # estimator: the telescoping sum of the level means (eq. MLMCestimator)
    exp = math.fsum(math.fsum(1.0 + vals[l][:x["drawn"]] - (1.0 if l else 0.0)) / x["drawn"]
                    for l, x in enumerate(r["levels"]))
    assert r["mean"] == pytest.approx(exp, rel=1e-14)


def _lib_or_skip():
    from paper_1903_08741_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("librmg.so not built (run __graft_entry__.build())")
    import paper_1903_08741_amd as rmg
    return rmg


def test_library_eq_mlmcsamp_matches_oracle():
    rmg = _lib_or_skip()
    rng = np.random.default_rng(11)
    for _ in range(200):
        L = int(rng.integers(1, 17))
        V = rng.uniform(0, 1, L) * 10.0 ** rng.uniform(-8, 0, L)
        Wl = rng.uniform(0.1, 1, L) * 10.0 ** rng.uniform(0, 6, L)
        eps = 10.0 ** rng.uniform(-4, -1)
        assert rmg.optimal_samples(eps, V, Wl) == list(mlmc.optimal_samples(eps, V, Wl))
    assert rmg.optimal_samples(0.1, [0.0, 1.0], [1.0, 2.0])[0] == 0


@pytest.mark.parametrize("V,W,eps", [([1.0], [0.0], 0.1), ([-1.0], [1.0], 0.1), ([1.0], [1.0], 0.0),
                                     ([1.0], [1.0], float("nan")), ([1e30], [1e-30], 1e-10), ([1.0] * 17, [1.0] * 17, 0.1)])
def test_library_eq_mlmcsamp_rejects_bad_input(V, W, eps):
    rmg = _lib_or_skip()
    with pytest.raises(rmg.RmgError):
        rmg.optimal_samples(eps, V, W)


def test_bias_uses_the_finest_parameter_set_on_both_grids():
    """Case C's hierarchy with continuation at the top: the finest level's own pairs
    (Y1 = 0, 0.2, ...) mix the parameter change into Y; the bias of eq. discErr (s = 2,
    a = 1) comes from further pairs of level 1 with Theta_L on both grids, numbered after
    the level's pairs: differences 0.03, -0.04 (the second of three draws fails) give
    sqrt((0.03^2 + 0.04^2) / 2) / (2 - 1) = 0.035355...; N_L = 2 such pairs are taken.
    Without a bias_pair source the level's own pairs give sqrt(mean Y1^2) = sqrt(0.02)."""
    def s(l, i):
        if l == 0:
            return (float(2 * (i % 2)), None, 1, 0)
        return (1.0 + 0.2 * (i % 2), 1.0, 1, 1)

    asked = []

    def bp(i):
        asked.append(i)
        k = len(asked) - 1
        return [(1.03, 1.0), (np.nan, 1.0), (0.96, 1.0)][k]

    r = pc_mlmc.run(s, [(2, 0), (5, 2)], [2, 2], 0.5, bias_pair=bp)
    assert r["levels"][1]["drawn"] == 2 and asked == [2, 3, 4] and r["bias_pairs"] == 3
    assert r["bias"] == pytest.approx(math.sqrt((0.03 ** 2 + 0.04 ** 2) / 2), rel=1e-12)
    r0 = pc_mlmc.run(s, [(2, 0), (5, 2)], [2, 2], 0.5)
    assert r0["bias"] == pytest.approx(math.sqrt(0.02), rel=1e-12) and r0["bias_pairs"] == 0
