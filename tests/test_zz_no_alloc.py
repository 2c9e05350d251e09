"""The allocation-free entry point picard_mg_solve_noalloc against picard_mg_solve (collected last).

Both run the same kernels on the same inputs, so results agree bit for bit (pressure
head, QoI, status, statistics).  Two calls in a row on the fixed scratch array, the second
with a smaller input (fewer samples, a smaller grid), so the second reads nothing the
first left behind; a call whose workspace exceeds the array is rejected with RMG_EINVAL.
Called through the C ABI with caller-allocated outputs.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_common import oracle_basis, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1903_08741_amd as rmg  # noqa: E402
from paper_1903_08741_amd import _abi  # noqa: E402

DEV = torch.device("cuda:0")


def _fields(n, S, wid):
    B = oracle_basis()[n]
    xi = W.xi_draws(wid, 0, range(S), 1, B.shape[0])
    return rmg.sample_fields(n, torch.from_numpy(B).to(DEV), torch.from_numpy(xi).to(DEV), [(0.0, 0.0, 1.0)])


def _call(ctx, fn, n, fields, prob, opts):
    S = fields.shape[0]
    h = torch.full((S, n * n), float("nan"), dtype=torch.float64, device=DEV)
    q = torch.full((S,), float("nan"), dtype=torch.float64, device=DEV)
    st = torch.full((S,), -7, dtype=torch.int32, device=DEV)
    stats = torch.zeros((S, C.sizeof(_abi.SampleStats)), dtype=torch.uint8, device=DEV)
    pr, op = prob.c(), opts.c()
    rc = fn(ctx._h, n, C.byref(pr), C.byref(op), C.c_void_p(fields.data_ptr()), S, C.c_void_p(h.data_ptr()),
            C.c_void_p(q.data_ptr()), C.c_void_p(st.data_ptr()), C.c_void_p(stats.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, h, q, st, stats


@pytest.mark.parametrize("precision", [rmg.FP64, rmg.MIXED])
def test_noalloc_equals_picard_mg_solve_two_calls(precision):
    ctx = rmg.Context(0)
    L = ctx._lib
    opts = rmg.SolverOpts(precision=precision, max_picard=25, fallback_cycles=2, fallback_max_picard=300)
    prob = rmg.Problem(n_steps=2)
    # first call 128^2 x 6 (streaming levels, fallback), then a smaller one 64^2 x 3, then 16^2 x 5
    for n, S, wid in ((128, 6, 50), (64, 3, 51), (16, 5, 52)):
        say(f"noalloc n={n} S={S} precision={precision}")
        fields = _fields(n, S, wid)
        ref = _call(ctx, L.picard_mg_solve, n, fields, prob, opts)
        got = _call(ctx, L.picard_mg_solve_noalloc, n, fields, prob, opts)
        assert got[0] == ref[0] and ref[0] in (0, rmg.RMG_ENOTCONV)
        for a, b in zip(got[1:], ref[1:]):
            assert torch.equal(torch.nan_to_num(a, nan=123.0), torch.nan_to_num(b, nan=123.0))
    ctx.close()


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    say("noalloc size limit")
    ctx = rmg.Context(0)
    n, S = 1024, 16   # ~2.3 GB of workspace
    fields = torch.ones((S, 1, n * n), dtype=torch.float64, device=DEV)
    rc, *_ = _call(ctx, ctx._lib.picard_mg_solve_noalloc, n, fields, rmg.Problem(n_steps=1), rmg.SolverOpts())
    assert rc == rmg.RMG_EINVAL
    assert b"scratch" in ctx._lib.rmg_last_error(ctx._h)
    ctx.close()
