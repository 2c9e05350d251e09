"""GPU parity for the fallback attempt, the error paths, the persisted tune cache and the
benchmark's largest grids.

  * Fallback: a sample that fails its first attempt restarts from its initial state with
    two cycles per Picard step (the oracle twin follows the same rule): FP64 within 1e-10
    of the twin with the same Picard counts over both attempts, mixed precision within
    1e-8; the streaming path switches to two cycle slots per pass while samples of the
    same class stay on one cycle, and the result does not depend on when it switches.
  * A non-finite field value flags its sample RMG_SAMPLE_NONFINITE without iterating it
    (QoI NaN, the call returns RMG_ENOTCONV, the fallback does not retry it) and leaves
    every other sample bit for bit unchanged, on the whole-sample and the streaming path.
  * A workspace cap below what a call needs returns RMG_ENOMEM without allocating.
  * The tune cache written by one context is read by the next; results are unchanged.
  * 256^2 with the benchmark's class (the 16 finest draws of the 5-level workload, tiles
    autotuned): element-wise against the twin oracle, FP64 (three streaming levels) within
    1e-10 with the same Picard counts, mixed (two FP32 streaming levels) within 1e-8.
  * 512^2 and 1024^2 (the van Genuchten hierarchy's finest grids; too large for the CPU
    oracle): mixed precision against the FP64 path, within 1e-8.
"""
from __future__ import annotations

import functools
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import oracle_basis, oracle_fields, oracle_solve, rel_inf, say
from oracle import kl as okl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1903_08741_amd as rmg  # noqa: E402

DEV = torch.device("cuda:0")


def _fields(n, S, wid, level=0):
    B = oracle_basis()[n]
    xi = W.xi_draws(wid, level, range(S), 1, B.shape[0])
    f = rmg.sample_fields(n, torch.from_numpy(B).to(DEV), torch.from_numpy(xi).to(DEV), [(0.0, 0.0, 1.0)])
    return B, xi, f


# ------------------------------------------------------------------ fallback
@pytest.mark.parametrize("n,precision,tol", [(16, rmg.FP64, 1e-10), (32, rmg.MIXED, 1e-8), (64, rmg.FP64, 1e-10),
                                             (64, rmg.MIXED, 1e-8), (128, rmg.MIXED, 1e-8)])
def test_fallback_matches_twin_oracle(n, precision, tol):
    """max_picard = 25 makes some draws fail their first attempt (one V(2,2) per step); they
    restart with two cycles per step and at most 300 iterations."""
    S, steps = 4, 2
    say(f"fallback n={n} precision={precision}")
    B, xi, fields = _fields(n, S, wid=40)
    prob = rmg.Problem(n_steps=steps)
    opts = rmg.SolverOpts(precision=precision, max_picard=25, fallback_cycles=2, fallback_max_picard=300)
    out = rmg.picard_mg_solve(n, fields, prob, opts)
    torch.cuda.synchronize()
    h = out["h"].cpu().numpy()
    st = out["stats"]
    oopts = dict(W.SOLVER, max_picard=25, fallback_cycles=2, fallback_max_picard=300)
    attempts = []
    for s in range(S):
        r = oracle_solve(n, oracle_fields(B, xi[s, 0]), dict(W.GARDNER_INFILTRATION, n_steps=steps), oopts)
        assert (out["status"][s].item() == 0) == (r["status"] == 0), s
        assert int(st["attempts"][s]) == r["attempts"], s
        attempts.append(r["attempts"])
        if r["status"] != 0:
            continue
        assert rel_inf(h[s].reshape(n, n), r["p"]) < tol, s
        if precision == rmg.FP64:
            assert int(st["picard_its"][s]) == sum(r["picard"]), (s, int(st["picard_its"][s]), r["picard"])
            assert int(st["mg_cycles"][s]) == r["cycles"], s
    assert 2 in attempts, "no draw exercised the fallback"


def test_fallback_graph_eager_and_slot_switch_are_bitwise_equal():
    """Graph replay and eager launches switch a 128^2 class to two cycle slots per pass at
    different times; the kernels take each sample's cycles from its state, so both agree
    bit for bit, also with the class forced onto the streaming path at 64^2."""
    say("fallback graph vs eager")
    for n, flags in ((128, 0), (64, rmg.FLAG_FORCE_STREAMING | rmg.FLAG_COARSE_TOP_32)):
        _, _, fields = _fields(n, 6, wid=41)
        prob = rmg.Problem(n_steps=2)
        base = dict(max_picard=45, fallback_cycles=2, fallback_max_picard=300)
        a = rmg.picard_mg_solve(n, fields, prob, rmg.SolverOpts(flags=flags, **base))
        b = rmg.picard_mg_solve(n, fields, prob, rmg.SolverOpts(flags=flags | rmg.FLAG_EAGER, **base))
        torch.cuda.synchronize()
        assert torch.equal(a["h"], b["h"])
        assert (a["stats"]["picard_its"] == b["stats"]["picard_its"]).all()
        assert (a["stats"]["attempts"] == b["stats"]["attempts"]).all()
        assert (a["stats"]["attempts"] == 2).any()


def test_fallback_in_batched_levels_counts_retried_pairs():
    grids, samples = (16, 32, 64), (24, 8, 4)
    say("fallback in mlmc_level_estimate")
    Bs = oracle_basis()
    levels = []
    for l, (n, S) in enumerate(zip(grids, samples)):
        xi = torch.from_numpy(W.xi_draws(42, l, range(S), 1, 64)).to(DEV)
        levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, fine=rmg.Problem(n_steps=2),
                           coarse=rmg.Problem(n_steps=2), basis_fine=torch.from_numpy(Bs[n]).to(DEV),
                           basis_coarse=torch.from_numpy(Bs[n // 2]).to(DEV) if l else None, xi=xi))
    opts = rmg.SolverOpts(max_picard=25, fallback_cycles=2, fallback_max_picard=300)
    sums, q, rc = rmg.mlmc_level_estimate(levels, [(0.0, 0.0, 1.0)], opts, return_qoi=True)
    assert rc == 0
    assert all(s["n_failed"] == 0 for s in sums)
    assert sum(s["n_retried"] for s in sums) > 0
    # without the fallback the same draws fail: the retried pairs are the ones that would be lost
    sums0, _, rc0 = rmg.mlmc_level_estimate(levels, [(0.0, 0.0, 1.0)], rmg.SolverOpts(max_picard=25),
                                            return_qoi=True)
    assert rc0 == rmg.RMG_ENOTCONV
    assert [s["n_failed"] for s in sums0] == [s["n_retried"] for s in sums]


# ------------------------------------------------------------ error paths
@pytest.mark.parametrize("n", [16, 128])
def test_nonfinite_field_flags_only_its_sample(n):
    S = 3
    say(f"non-finite field n={n}")
    _, _, fields = _fields(n, S, wid=43)
    prob = rmg.Problem(n_steps=2)
    opts = rmg.SolverOpts(max_picard=500)
    clean = rmg.picard_mg_solve(n, fields, prob, opts)
    assert (clean["status"] == 0).all()
    bad = fields.clone()
    bad[1, 0, (n * n) // 2 + 3] = float("nan")
    out = rmg.picard_mg_solve(n, bad, prob, opts)
    torch.cuda.synchronize()
    assert out["rc"] == rmg.RMG_ENOTCONV
    st = out["status"].cpu().numpy()
    assert st[1] == rmg.SAMPLE_NONFINITE and st[0] == 0 and st[2] == 0
    assert torch.isnan(out["qoi"][1])
    for s in (0, 2):
        assert torch.equal(out["h"][s], clean["h"][s])
        assert out["qoi"][s].item() == clean["qoi"][s].item()
    assert int(out["stats"]["picard_its"][1]) == 0  # validated, never iterated
    # invalid input is not retried by the fallback
    fb = rmg.picard_mg_solve(n, bad, prob, rmg.SolverOpts(max_picard=500, fallback_cycles=2,
                                                          fallback_max_picard=100))
    assert fb["status"][1].item() == rmg.SAMPLE_NONFINITE and int(fb["stats"]["attempts"][1]) == 1


def test_workspace_limit_returns_enomem():
    say("workspace limit")
    ctx = rmg.Context(0)
    _, _, fields = _fields(128, 4, wid=44)
    prob, opts = rmg.Problem(n_steps=1), rmg.SolverOpts()
    ctx.set_workspace_limit(1 << 20)
    with pytest.raises(rmg.RmgError) as e:
        ctx.picard_mg_solve(128, fields, prob, opts)
    assert e.value.code == rmg.RMG_ENOMEM
    ctx.set_workspace_limit(0)
    out = ctx.picard_mg_solve(128, fields, prob, opts)
    assert out["rc"] in (0, rmg.RMG_ENOTCONV)  # solved (a draw may exceed the iteration limit)
    ctx.close()


def test_tune_cache_is_persisted_and_reused(tmp_path):
    say("tune cache")
    path = str(tmp_path / "rmg_tune.txt")
    _, _, fields = _fields(128, 3, wid=45)
    prob, opts = rmg.Problem(n_steps=1), rmg.SolverOpts()
    c1 = rmg.Context(0, tune_cache=path)
    a = c1.picard_mg_solve(128, fields, prob, opts)
    torch.cuda.synchronize()
    choices = c1.tune_choices()
    c1.close()
    text = open(path).read()
    assert "tiles n=128 S=3" in text and "gfx" in text
    assert os.listdir(tmp_path) == ["rmg_tune.txt"]  # the context's temporary copy was renamed
    # the context reports the same choices as the file holds (device key stripped)
    lines = [ln.split("\t") for ln in text.splitlines()]
    assert len(choices) == len(lines) >= 1
    for key, val in lines:
        assert choices[key[key.index("] ") + 2:]] == val
    mtime = os.path.getmtime(path)
    c2 = rmg.Context(0, tune_cache=path)
    b = c2.picard_mg_solve(128, fields, prob, opts)
    torch.cuda.synchronize()
    c2.close()
    assert torch.equal(a["h"], b["h"])
    assert os.path.getmtime(path) == mtime  # nothing new to tune


# ---------------------------------------------------- 256^2 benchmark class
@functools.lru_cache(maxsize=None)
def _benchmark_256():
    f = W.KS_FIELD
    _, B = okl.basis(f["sigma2"], f["corr_len"], f["n_modes"], [256], ref_n=64)
    return B[256]


@functools.lru_cache(maxsize=None)
def _oracle_256(i):
    B = _benchmark_256()
    xi = W.xi_draws(W.MLMC_5LEVEL["workload_id"], 4, [i], 1, 64)[0, 0]
    say(f"oracle 256^2 draw {i}")
    return oracle_solve(256, oracle_fields(B, xi), dict(W.GARDNER_INFILTRATION, n_steps=2),
                        dict(W.SOLVER, max_picard=500))


@pytest.mark.parametrize("precision,tol", [(rmg.FP64, 1e-10), (rmg.MIXED, 1e-8)])
def test_256_benchmark_class_elementwise(precision, tol):
    """The 256^2 grid-size class of the benchmark call (its 16 draws; autotuned tiles),
    two steps; draws 0 and 8 converge in both steps with one V(2,2) per Picard step."""
    say(f"256^2 benchmark class precision={precision}")
    B = _benchmark_256()
    xi = W.xi_draws(W.MLMC_5LEVEL["workload_id"], 4, range(16), 1, 64)
    fields = rmg.sample_fields(256, torch.from_numpy(B).to(DEV), torch.from_numpy(xi).to(DEV),
                               [(0.0, W.KS_FIELD["log_mean"], W.KS_FIELD["scale"])])
    out = rmg.picard_mg_solve(256, fields, rmg.Problem(n_steps=2), rmg.SolverOpts(precision=precision,
                                                                                   max_picard=500))
    torch.cuda.synchronize()
    h = out["h"].cpu().numpy()
    for i in (0, 8):
        r = _oracle_256(i)
        assert r["status"] == 0 and out["status"][i].item() == 0
        assert rel_inf(h[i].reshape(256, 256), r["p"]) < tol, i
        if precision == rmg.FP64:
            assert int(out["stats"]["picard_its"][i]) == sum(r["picard"]), (i, r["picard"])


# -------------------------------------------- 512^2 and 1024^2, mixed vs FP64
@pytest.mark.parametrize("n,S", [(512, 2), (1024, 1)])
def test_large_grid_mixed_matches_fp64(n, S):
    """The van Genuchten infiltration problem of the largest grids (three KL fields, the
    finest level's parameters), two steps: the mixed-precision path against the FP64 path."""
    from paper_1903_08741_amd import kl_setup
    say(f"{n}^2 mixed vs FP64")
    vf, tw = W.VG_FIELDS, W.VG_INFILTRATION
    _, tables = kl_setup.kl_tables(1.0, vf["corr_len"], vf["n_modes"], [n])
    xi = W.xi_draws(46, 0, range(S), 3, vf["n_modes"])
    fields = rmg.sample_fields(n, torch.from_numpy(tables[n]).to(DEV), torch.from_numpy(xi).to(DEV),
                               list(vf["marginals"]))
    prob = rmg.Problem(model=rmg.VGM, n_steps=2, theta_r=tw["theta_r"], theta_s=tw["theta_s"], h_top=tw["h_top"],
                       h_bottom=tw["h_bottom"], h_init=tw["h_init"], dt=tw["dt"], init_profile=1,
                       init_rate=tw["init_rate"])
    a = rmg.picard_mg_solve(n, fields, prob, rmg.SolverOpts(precision=rmg.MIXED, max_picard=200))
    b = rmg.picard_mg_solve(n, fields, prob, rmg.SolverOpts(precision=rmg.FP64, max_picard=200))
    torch.cuda.synchronize()
    assert (a["status"] == 0).all() and (b["status"] == 0).all()
    for s in range(S):
        err = rel_inf(a["h"][s].cpu().numpy(), b["h"][s].cpu().numpy())
        say(f"  sample {s}: rel err {err:.2e}, its {int(a['stats']['picard_its'][s])} / "
            f"{int(b['stats']['picard_its'][s])}")
        assert err < 1e-8, s
