"""Batched Picard-multigrid sampler for the stochastic Richards equation on MI355X.

Python binding of the C ABI in include/rmg.h (argument marshalling only; every
step of the computation runs in the HIP kernels of librmg.so).  Device memory and
streams come from PyTorch: arrays are torch CUDA tensors (ROCm) and work is
enqueued on the current torch stream.

    sample_fields(n, basis, xi, marginals)           KL fields (Section 3)
    picard_mg_solve(n, fields, problem, opts)        S samples on one grid (Sections 4.1-4.2)
    mlmc_level_estimate(levels, marginals, opts)     batched MLMC level sums (Section 5.1)
    pc_mlmc(levels, marginals, opts, eps, xi_source) adaptive PC_MLMC (Section 5.1, Algorithm 1)
    picard_mg_adjoint(n, basis, xi, marginal, ...)   outflux QoI and dQ/dxi by the discrete adjoint
    outflux_qoi(xi, basis, n, marginal, ...)         the same as a torch.autograd.Function
    optimal_samples(eps, V, W)                       eq. MLMCSAMP (host)
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field, fields as dc_fields

from . import _abi
from ._abi import (COST_TIME, COST_WORK, CYCLE_V, CYCLE_W, FLAG_COARSE_TOP_32, FLAG_CONFINE, FLAG_EAGER, FLAG_FORCE_STREAMING, FLAG_NO_AUTOTUNE,  # noqa: F401
                   FLAG_NO_CONFINE, FLAG_STATE_GLOBAL, FLAG_TILES_16, FLAG_WHOLE_WHERE_FITS, FP64, GARDNER, LINEAR,
                   MIXED, QOI_MEAN_SATURATION, RMG_EINVAL, RMG_ENOMEM, RMG_ENOTCONV, RMG_OK, SAMPLE_MAXITER,
                   SAMPLE_NONFINITE, SAMPLE_OK, TIME_COARSE, TIME_FINE, TIME_NONE, TIME_SMOOTHER_DOWN, VGM)

__all__ = ["Problem", "SolverOpts", "Context", "RmgError", "sample_fields", "picard_mg_solve",
           "mlmc_level_estimate", "pc_mlmc", "optimal_samples", "picard_mg_adjoint", "outflux_qoi",
           "default_context"]


class RmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rmg error {code}: {msg}")
        self.code = code


@dataclass
class Problem:
    """Deterministic problem data (mirrors rmg_problem)."""
    model: int = GARDNER
    n_steps: int = 10
    qoi: int = QOI_MEAN_SATURATION
    theta_r: float = 0.05
    theta_s: float = 0.5
    gardner_a: float = 1.0
    linear_c0: float = 0.0
    vg_alpha_shift: float = 0.0
    vg_n_shift: float = 0.0
    h_top: float = 0.0
    h_bottom: float = -10.0
    h_init: float = -10.0
    dt: float = 0.01
    init_profile: int = 0
    init_rate: float = 0.0

    def c(self) -> _abi.Problem:
        return _abi.Problem(**{f.name: getattr(self, f.name) for f in dc_fields(self)})

    @property
    def n_fields(self) -> int:
        return 3 if self.model == VGM else 1


@dataclass
class SolverOpts:
    """Solver options (mirrors rmg_solver_opts)."""
    precision: int = MIXED
    cycle: int = CYCLE_V
    nu1: int = 2
    nu2: int = 2
    cycles_per_picard: int = 1
    max_picard: int = 100
    coarsest_n: int = 4
    flags: int = 0
    fallback_cycles: int = 0
    fallback_max_picard: int = 0
    eps_mg: float = 1e-5
    eps_picard: float = 1e-8

    def c(self) -> _abi.SolverOpts:
        return _abi.SolverOpts(**{f.name: getattr(self, f.name) for f in dc_fields(self)})


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_dev(t, name, dtype=None, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """An rmg_ctx on one HIP device (owns the workspace and its streams).

    A context is not thread safe.  Separate contexts are independent: calls on different
    contexts from different threads overlap on the GPU and return the results of the same
    calls made one at a time (mlmc_level_estimate calls made so should pass
    FLAG_NO_CONFINE; two contexts per device measured best)."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        """tune_cache: optional file that persists the autotuner's choices across processes."""
        self._lib = _abi.lib()
        h = C.c_void_p()
        rc = self._lib.rmg_ctx_create(C.byref(h), int(device), tune_cache.encode() if tune_cache else None)
        if rc != RMG_OK:
            raise RmgError(rc, f"rmg_ctx_create(device={device}) failed")
        self._h = h
        self.device = device

    def set_workspace_limit(self, nbytes: int):
        """Cap the context's workspace (0: no cap); calls that would exceed it raise RMG_ENOMEM."""
        self._raise(self._lib.rmg_ctx_set_workspace_limit(self._h, int(nbytes)))

    def tune_text(self) -> str:
        """The context's tuning choices in the tune-cache file's format (rmg_ctx_tune_dump):
        written to a file and given to a new context, they start it tuned."""
        n = self._lib.rmg_ctx_tune_dump(self._h, None, 0)
        if n < 0:
            self._raise(int(n))
        buf = C.create_string_buffer(int(n) + 1)
        self._lib.rmg_ctx_tune_dump(self._h, buf, int(n) + 1)
        return buf.value.decode()

    def tune_choices(self):
        """The context's tuning choices: {signature: choice} (tile edges per streaming class
        signature "tiles ...", "confine passes" per batched-call signature "sched ...")."""
        out = {}
        for line in self.tune_text().splitlines():
            k, _, v = line.partition("\t")
            i = k.find("] ")  # drop the device key "[arch cu=N] "
            out[k[i + 2:] if k.startswith("[") and i >= 0 else k] = v
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rmg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, rc, allow_notconv=False):
        if rc == RMG_OK or (allow_notconv and rc == RMG_ENOTCONV):
            return rc
        raise RmgError(rc, self._lib.rmg_last_error(self._h).decode())

    def set_kernel_timing(self, which: int):
        """Time the launches of the selected kernel kinds (a mask of ``TIME_*``) and reset the totals."""
        self._raise(self._lib.rmg_set_kernel_timing(self._h, int(which)))

    def kernel_timing(self, kind: int = TIME_SMOOTHER_DOWN) -> dict:
        """Totals of one kind since set_kernel_timing: launches, cells (work units), total_ms, algo_bytes."""
        t = _abi.KernelTiming()
        self._raise(self._lib.rmg_get_kernel_timing(self._h, int(kind), C.byref(t)))
        return {k: getattr(t, k) for k in ("launches", "cells", "total_ms", "algo_bytes")}

    # -- entry points ----------------------------------------------------------
    def sample_fields(self, n, basis, xi, marginals, out=None, stream=None):
        """KL fields [S][F][n*n] from basis [M][n*n] and standard normals xi [S][F][M] (FP64)."""
        torch = _torch()
        M = basis.shape[0]
        S, F = xi.shape[0], xi.shape[1]
        _check_dev(basis, "basis", torch.float64, (M, n * n))
        _check_dev(xi, "xi", torch.float64, (S, F, M))
        if len(marginals) != F:
            raise ValueError("one marginal per field is required")
        if out is None:
            out = torch.empty((S, F, n * n), dtype=torch.float64, device=xi.device)
        _check_dev(out, "out", torch.float64, (S, F, n * n))
        marg = (_abi.Marginal * F)(*[_abi.Marginal(*m) for m in marginals])
        rc = self._lib.sample_fields(self._h, n, F, M, C.c_void_p(basis.data_ptr()),
                                     C.c_void_p(xi.data_ptr()), marg, S, C.c_void_p(out.data_ptr()),
                                     _stream_ptr(stream))
        self._raise(rc)
        return out

    def picard_mg_solve(self, n, fields, problem: Problem, opts: SolverOpts, stream=None, noalloc=False):
        """Solve S samples on an n x n grid; returns dict(h, qoi, status, stats, rc).
        noalloc: the allocation-free entry point (workspace in the library's fixed device array)."""
        torch = _torch()
        S = fields.shape[0]
        _check_dev(fields, "fields", torch.float64, (S, problem.n_fields, n * n))
        dev = fields.device
        h = torch.empty((S, n * n), dtype=torch.float64, device=dev)
        qoi = torch.empty(S, dtype=torch.float64, device=dev)
        status = torch.empty(S, dtype=torch.int32, device=dev)
        stats = torch.empty((S, C.sizeof(_abi.SampleStats)), dtype=torch.uint8, device=dev)
        pr, op = problem.c(), opts.c()
        fn = self._lib.picard_mg_solve_noalloc if noalloc else self._lib.picard_mg_solve
        rc = fn(self._h, n, C.byref(pr), C.byref(op), C.c_void_p(fields.data_ptr()),
                                       S, C.c_void_p(h.data_ptr()), C.c_void_p(qoi.data_ptr()),
                                       C.c_void_p(status.data_ptr()), C.c_void_p(stats.data_ptr()),
                                       _stream_ptr(stream))
        self._raise(rc, allow_notconv=True)
        return dict(h=h, qoi=qoi, status=status, stats=_decode_stats(stats), rc=rc)

    def mlmc_level_estimate(self, levels, marginals, opts: SolverOpts, return_qoi=False, stream=None):
        """levels: list of dict(n_fine, n_coarse, fine: Problem, coarse: Problem|None,
        basis_fine, basis_coarse, xi); returns (list of per-level sums dicts, qoi tensor|None, rc)."""
        torch = _torch()
        L = len(levels)
        arr = (_abi.Level * L)()
        F = levels[0]["xi"].shape[1]
        M = levels[0]["xi"].shape[2]
        tot = 0
        for i, lv in enumerate(levels):
            S = lv["xi"].shape[0]
            _check_dev(lv["xi"], f"levels[{i}].xi", torch.float64, (S, F, M))
            _check_dev(lv["basis_fine"], f"levels[{i}].basis_fine", torch.float64,
                       (M, lv["n_fine"] ** 2))
            coarse = lv.get("coarse") or lv["fine"]
            bc = lv.get("basis_coarse")
            if lv["n_coarse"]:
                _check_dev(bc, f"levels[{i}].basis_coarse", torch.float64, (M, lv["n_coarse"] ** 2))
            arr[i] = _abi.Level(lv["n_fine"], lv["n_coarse"], S, lv["fine"].c(), coarse.c(),
                                C.c_void_p(lv["basis_fine"].data_ptr()),
                                C.c_void_p(bc.data_ptr()) if bc is not None else None,
                                C.c_void_p(lv["xi"].data_ptr()))
            tot += 2 * S
        marg = (_abi.Marginal * F)(*[_abi.Marginal(*m) for m in marginals])
        out = (_abi.LevelSums * L)()
        q = torch.empty(tot, dtype=torch.float64, device=levels[0]["xi"].device) if return_qoi else None
        op = opts.c()
        rc = self._lib.mlmc_level_estimate(self._h, L, arr, F, M, marg, C.byref(op), out,
                                           C.c_void_p(q.data_ptr()) if q is not None else None,
                                           _stream_ptr(stream))
        self._raise(rc, allow_notconv=True)
        return [_decode_sums(s) for s in out], q, rc

    def picard_mg_adjoint(self, n, basis, xi, marginal, problem: Problem, opts: SolverOpts, ckpt_every=1,
                          eps_adjoint=1e-12, stream=None):
        """Time-integrated bottom outflux Q per sample and dQ/dxi by the discrete adjoint.
        basis [M][n*n], xi [S][M] float64 device tensors; marginal (shift, log_mean, scale) of Ks.
        Returns dict(q [S], grad [S][M], status [S], stats_forward, stats_adjoint, rc)."""
        torch = _torch()
        S, M = xi.shape
        _check_dev(xi, "xi", torch.float64, (S, M))
        _check_dev(basis, "basis", torch.float64, (M, n * n))
        dev = xi.device
        q = torch.empty(S, dtype=torch.float64, device=dev)
        grad = torch.empty(S, M, dtype=torch.float64, device=dev)
        status = torch.empty(S, dtype=torch.int32, device=dev)
        stats = torch.empty(2 * S * C.sizeof(_abi.SampleStats), dtype=torch.uint8, device=dev)
        pr = problem.c()
        pr.qoi = _abi.QOI_BOTTOM_OUTFLUX
        op = opts.c()
        mg = _abi.Marginal(*marginal)
        rc = self._lib.picard_mg_adjoint(self._h, int(n), C.byref(pr), C.byref(op), int(M),
                                         C.c_void_p(basis.data_ptr()), C.byref(mg), C.c_void_p(xi.data_ptr()),
                                         int(S), int(ckpt_every), float(eps_adjoint), C.c_void_p(q.data_ptr()),
                                         C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()),
                                         C.c_void_p(stats.data_ptr()), _stream_ptr(stream))
        self._raise(rc, allow_notconv=True)
        st = _decode_stats(stats)
        return dict(q=q, grad=grad, status=status, stats_forward=st[:S], stats_adjoint=st[S:], rc=rc)

    def picard_mg_outflux(self, n, basis, xi, marginal, problem: Problem, opts: SolverOpts, stream=None):
        """Time-integrated bottom outflux Q per sample by the forward solve alone (the Q of
        picard_mg_adjoint, bit for bit).  Returns dict(q [S], status [S], stats, rc)."""
        torch = _torch()
        S, M = xi.shape
        _check_dev(xi, "xi", torch.float64, (S, M))
        _check_dev(basis, "basis", torch.float64, (M, n * n))
        dev = xi.device
        q = torch.empty(S, dtype=torch.float64, device=dev)
        status = torch.empty(S, dtype=torch.int32, device=dev)
        stats = torch.empty(S * C.sizeof(_abi.SampleStats), dtype=torch.uint8, device=dev)
        pr = problem.c()
        pr.qoi = _abi.QOI_BOTTOM_OUTFLUX
        op = opts.c()
        mg = _abi.Marginal(*marginal)
        rc = self._lib.picard_mg_outflux(self._h, int(n), C.byref(pr), C.byref(op), int(M),
                                         C.c_void_p(basis.data_ptr()), C.byref(mg), C.c_void_p(xi.data_ptr()),
                                         int(S), C.c_void_p(q.data_ptr()), C.c_void_p(status.data_ptr()),
                                         C.c_void_p(stats.data_ptr()), _stream_ptr(stream))
        self._raise(rc, allow_notconv=True)
        return dict(q=q, status=status, stats=_decode_stats(stats), rc=rc)

    def pc_mlmc(self, levels, marginals, opts: SolverOpts, eps: float, xi_source, bias_rate=1.0,
                cost_model=_abi.COST_WORK, max_rounds=50, max_pairs=1 << 40, max_pairs_per_call=0,
                stream=None):
        """Adaptive PC_MLMC (Algorithm 1).  levels: list of dict(n_fine, n_coarse, n_warmup,
        fine: Problem, coarse: Problem|None, basis_fine, basis_coarse); xi_source(level, first,
        count) returns a float64 array [count][n_fields][n_modes] of standard normals.
        Returns dict(levels=[per-level dicts], mean, var, sampling_err2, bias, total_cost,
        wall_ms, rounds, converged, calls, rc)."""
        import numpy as np
        torch = _torch()
        L = len(levels)
        F = len(marginals)
        M = levels[0]["basis_fine"].shape[0]
        arr = (_abi.PcLevel * L)()
        for i, lv in enumerate(levels):
            _check_dev(lv["basis_fine"], f"levels[{i}].basis_fine", torch.float64, (M, lv["n_fine"] ** 2))
            bc = lv.get("basis_coarse")
            if lv["n_coarse"]:
                _check_dev(bc, f"levels[{i}].basis_coarse", torch.float64, (M, lv["n_coarse"] ** 2))
            coarse = lv.get("coarse") or lv["fine"]
            arr[i] = _abi.PcLevel(lv["n_fine"], lv["n_coarse"], int(lv["n_warmup"]), lv["fine"].c(), coarse.c(),
                                  C.c_void_p(lv["basis_fine"].data_ptr()),
                                  C.c_void_p(bc.data_ptr()) if bc is not None else None)
        failure = []

        def _src(_user, level, first, count, h_xi):
            try:
                x = np.ascontiguousarray(xi_source(level, first, count), dtype=np.float64)
                if x.shape != (count, F, M):
                    raise ValueError(f"xi_source returned shape {x.shape}, expected {(count, F, M)}")
                C.memmove(h_xi, x.ctypes.data, x.nbytes)
                return 0
            except BaseException as e:  # reported after the call returns
                failure.append(e)
                return 1

        cb = _abi.XiSource(_src)
        marg = (_abi.Marginal * F)(*[_abi.Marginal(*m) for m in marginals])
        po = _abi.PcOpts(float(eps), float(bias_rate), int(cost_model), int(max_rounds), int(max_pairs),
                         int(max_pairs_per_call))
        lout = (_abi.PcLevelOut * L)()
        res = _abi.PcResult()
        op = opts.c()
        rc = self._lib.pc_mlmc(self._h, L, arr, F, M, marg, C.byref(op), C.byref(po), cb, None, lout,
                               C.byref(res), _stream_ptr(stream))
        if failure:
            raise failure[0]
        self._raise(rc, allow_notconv=True)
        out = {k: getattr(res, k) for k in ("mean", "var", "sampling_err2", "bias", "total_cost", "wall_ms",
                                            "rounds", "converged", "calls", "bias_pairs")}
        out["levels"] = [dict(drawn=o.drawn, target=o.target, W=o.W, V=o.V, mean=o.mean,
                              sums=_decode_sums(o.sums)) for o in lout]
        out["rc"] = rc
        return out


def _decode_sums(s) -> dict:
    d = {k: getattr(s, k) for k in ("n", "n_failed", "picard_its", "mg_cycles", "mg_cycles_coarse", "n_retried")}
    for k in ("sY", "sY2", "sQf", "sQf2", "sQc", "sQc2"):
        v = getattr(s, k)
        d[k] = (v.hi, v.lo)
    return d


def optimal_samples(eps, V, W):
    """Eq. MLMCSAMP evaluated by the library (host arithmetic; no device needed)."""
    L = len(V)
    Va, Wa, N = (C.c_double * L)(*V), (C.c_double * L)(*W), (C.c_int64 * L)()
    rc = _abi.lib().rmg_mlmc_optimal_samples(L, Va, Wa, float(eps), N)
    if rc != RMG_OK:
        raise RmgError(rc, "rmg_mlmc_optimal_samples: invalid arguments")
    return list(N)


def _decode_stats(raw):
    import numpy as np
    a = raw.cpu().numpy()
    dt = np.dtype([("picard_its", "<i4"), ("mg_cycles", "<i4"), ("steps_done", "<i4"), ("status", "<i4"),
                   ("final_dp_inf", "<f8"), ("attempts", "<i4"), ("reserved", "<i4")])
    return a.view(dt).reshape(-1)


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def sample_fields(n, basis, xi, marginals, out=None, stream=None):
    return default_context(xi.device.index or 0).sample_fields(n, basis, xi, marginals, out, stream)


def picard_mg_solve(n, fields, problem: Problem, opts: SolverOpts, stream=None):
    return default_context(fields.device.index or 0).picard_mg_solve(n, fields, problem, opts, stream)


def mlmc_level_estimate(levels, marginals, opts: SolverOpts, return_qoi=False, stream=None):
    dev = levels[0]["xi"].device.index or 0
    return default_context(dev).mlmc_level_estimate(levels, marginals, opts, return_qoi, stream)


def picard_mg_adjoint(n, basis, xi, marginal, problem: Problem, opts: SolverOpts, **kw):
    return default_context(xi.device.index or 0).picard_mg_adjoint(n, basis, xi, marginal, problem, opts, **kw)


def _make_outflux_fn():
    torch = _torch()

    class OutfluxFn(torch.autograd.Function):
        """Q(xi) = time-integrated bottom outflux of every sample, differentiable in xi.

        The forward pass is the forward solve alone (picard_mg_outflux); the backward pass
        runs the discrete adjoint (picard_mg_adjoint: forward with checkpoints, then the
        adjoint sweep) for the saved inputs and scales dQ/dxi by the incoming gradient.  A
        forward under torch.no_grad() therefore costs one forward solve."""

        @staticmethod
        def forward(ctx, xi, basis, n, marginal, problem, opts, ckpt_every, eps_adjoint):
            xd = xi.detach().contiguous()
            dev = xd.device.index or 0
            out = default_context(dev).picard_mg_outflux(n, basis, xd, marginal, problem, opts)
            ctx.save_for_backward(xd, basis)
            ctx.args = (n, marginal, problem, opts, ckpt_every, eps_adjoint)
            ctx.status = out["status"]
            return out["q"]

        @staticmethod
        def backward(ctx, gq):
            xd, basis = ctx.saved_tensors
            n, marginal, problem, opts, ckpt_every, eps_adjoint = ctx.args
            out = picard_mg_adjoint(n, basis, xd, marginal, problem, opts, ckpt_every=ckpt_every,
                                    eps_adjoint=eps_adjoint)
            return gq[:, None] * out["grad"], None, None, None, None, None, None, None

    return OutfluxFn


_OUTFLUX_FN = None


def outflux_qoi(xi, basis, n, marginal, problem: Problem, opts: SolverOpts, ckpt_every=1, eps_adjoint=1e-12):
    """Differentiable time-integrated bottom outflux (torch.autograd.Function over the adjoint)."""
    global _OUTFLUX_FN
    if _OUTFLUX_FN is None:
        _OUTFLUX_FN = _make_outflux_fn()
    return _OUTFLUX_FN.apply(xi, basis, n, marginal, problem, opts, ckpt_every, eps_adjoint)


def pc_mlmc(levels, marginals, opts: SolverOpts, eps: float, xi_source, **kw):
    dev = levels[0]["basis_fine"].device.index or 0
    return default_context(dev).pc_mlmc(levels, marginals, opts, eps, xi_source, **kw)
