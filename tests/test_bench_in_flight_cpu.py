"""Host logic of bench.py's steps in flight (no GPU): how the timed steps are dealt out over
the contexts, that the contexts' calls really run at the same time, that every result is
returned, that an error in one thread reaches the caller, and the bitwise result check."""
import contextlib
import threading

import pytest

import bench

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("steps,P,want", [(6, 2, [3, 3]), (5, 2, [3, 2]), (1, 2, [1, 0]), (7, 3, [3, 2, 2])])
def test_in_flight_counts(steps, P, want):
    assert bench.in_flight_counts(steps, P) == want
    assert sum(bench.in_flight_counts(steps, P)) == steps


def test_calls_of_two_contexts_overlap_and_all_results_return():
    meet = threading.Barrier(2, timeout=10)  # breaks (and fails the test) if the calls run one by one

    def call(ctx):
        meet.wait()
        ctx["n"] += 1
        return ctx["id"], ctx["n"]

    ctxs = [{"id": 0, "n": 0}, {"id": 1, "n": 0}]
    out = bench.run_in_flight(torch, ctxs, 4, call, on_stream=contextlib.nullcontext)
    assert sorted(out) == [(0, 1), (0, 2), (1, 1), (1, 2)]


def test_error_in_one_context_reaches_the_caller():
    def call(ctx):
        if ctx == 1:
            raise RuntimeError("call failed")
        return ctx

    with pytest.raises(RuntimeError, match="call failed"):
        bench.run_in_flight(torch, [0, 1], 4, call, on_stream=contextlib.nullcontext)


def test_same_results_is_bitwise():
    q = torch.tensor([1.0, float("nan"), -0.0], dtype=torch.float64)
    sums = [{"n": 3, "sY": (1.0, 0.0)}]
    assert bench.same_results(torch, [(sums, q, 0), (list(sums), q.clone(), 0)])
    q2 = q.clone()
    q2[2] = 0.0  # -0.0 and 0.0 compare equal but differ in their bits
    assert not bench.same_results(torch, [(sums, q, 0), (sums, q2, 0)])
    assert not bench.same_results(torch, [(sums, q, 0), ([{"n": 3, "sY": (1.0, 1e-30)}], q, 0)])
