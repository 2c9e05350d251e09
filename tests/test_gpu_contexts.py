"""Calls on separate contexts from separate host threads (the header's concurrency
contract): two contexts, each driven by its own thread and torch stream, solve their
workloads at the same time, and every result equals, bit for bit, that of the same
call made alone on a third context.

Workloads: the Gardner MLMC estimator on 16^2..128^2 (whole-sample classes, streaming
classes, the coarse kernel) and the van Genuchten estimator with three fields on
16^2..32^2, whose 32^2 whole-sample launches need more LDS than the Gardner ones with
the same kernel (the per-kernel LDS limit is shared by the contexts).
"""
from __future__ import annotations

import threading

import pytest

import workloads as W
from gpu_common import oracle_basis, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1903_08741_amd as rmg  # noqa: E402

DEV = torch.device("cuda:0")


def gardner_job():
    Bs = oracle_basis()
    levels = []
    for l, (n, S) in enumerate(zip((16, 32, 64, 128), (8, 4, 3, 2))):
        xi = torch.from_numpy(W.xi_draws(23, l, range(S), 1, 64)).to(DEV)
        levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, fine=rmg.Problem(n_steps=3),
                           coarse=rmg.Problem(n_steps=3), basis_fine=torch.from_numpy(Bs[n]).to(DEV),
                           basis_coarse=torch.from_numpy(Bs[n // 2]).to(DEV) if l else None, xi=xi))
    return levels, [(0.0, 0.0, 1.0)], rmg.SolverOpts(precision=rmg.MIXED)


def vg_job():
    from oracle import kl as okl
    VF = W.VG_FIELDS
    _, B = okl.basis(1.0, VF["corr_len"], VF["n_modes"], [8, 16, 32], ref_n=32)
    g = W.VG_INFILTRATION
    prob = rmg.Problem(model=rmg.VGM, n_steps=2, theta_r=g["theta_r"], theta_s=g["theta_s"], h_top=g["h_top"],
                       h_bottom=g["h_bottom"], h_init=g["h_init"], dt=g["dt"], init_profile=1,
                       init_rate=g["init_rate"])
    levels = []
    for l, (n, S) in enumerate(zip((16, 32), (6, 4))):
        xi = torch.from_numpy(W.xi_draws(W.MLMC_VG["workload_id"], 30 + l, range(S), 3, VF["n_modes"])).to(DEV)
        levels.append(dict(n_fine=n, n_coarse=n // 2 if l else 0, fine=prob, coarse=prob,
                           basis_fine=torch.from_numpy(B[n]).to(DEV),
                           basis_coarse=torch.from_numpy(B[n // 2]).to(DEV) if l else None, xi=xi))
    return levels, list(VF["marginals"]), rmg.SolverOpts(precision=rmg.MIXED)


def solve(ctx, job):
    levels, marg, opts = job
    sums, q, _ = ctx.mlmc_level_estimate(levels, marg, opts, return_qoi=True)
    return sums, q.view(torch.int64).cpu()


def run_threads(jobs_per_thread):
    """One context, host thread and stream per entry; each thread makes its calls in order."""
    ctxs = [rmg.Context(0) for _ in jobs_per_thread]
    out = [[] for _ in jobs_per_thread]
    errs = []

    def worker(j):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for job in jobs_per_thread[j]:
                    out[j].append(solve(ctxs[j], job))
            st.synchronize()
        except BaseException as e:
            errs.append(e)

    th = [threading.Thread(target=worker, args=(j,)) for j in range(len(jobs_per_thread))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for c in ctxs:
        c.close()
    if errs:
        raise errs[0]
    return out


def test_concurrent_contexts_match_a_lone_context_bitwise():
    gj, vj = gardner_job(), vg_job()
    ref_ctx = rmg.Context(0)
    say("contexts: reference calls on one context")
    ref_g, ref_v = solve(ref_ctx, gj), solve(ref_ctx, vj)
    ref_ctx.close()
    say("contexts: two threads, Gardner twice against van Genuchten twice")
    got = run_threads([[gj, gj], [vj, vj]])
    for sums, q in got[0]:
        assert sums == ref_g[0] and torch.equal(q, ref_g[1])
    for sums, q in got[1]:
        assert sums == ref_v[0] and torch.equal(q, ref_v[1])
    say("contexts: two threads, the Gardner workload on both")
    got = run_threads([[gj, gj], [gj]])
    for row in got:
        for sums, q in row:
            assert sums == ref_g[0] and torch.equal(q, ref_g[1])
