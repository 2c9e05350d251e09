"""Helpers for the GPU parity tests: oracle references and device inputs.

Every expected value comes from the CPU oracle on the same seeded inputs; the
KL basis handed to the GPU is the oracle's own table (an input, not a result).
"""
from __future__ import annotations

import functools
import sys

import numpy as np

import workloads as W
from oracle import kl as okl, picard as opicard, qoi as oqoi


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def oracle_basis(grids=(4, 8, 16, 32, 64, 128), n_modes=64, ref_n=32):
    f = W.KS_FIELD
    lam, B = okl.basis(f["sigma2"], f["corr_len"], n_modes, list(grids), ref_n=ref_n)
    return B


def oracle_fields(B, xi_row):
    return okl.lognormal(okl.gaussian_field(xi_row, B), W.KS_FIELD["log_mean"], W.KS_FIELD["scale"])


def oracle_solve(n, Ks, prob: dict, opts: dict):
    r = opicard.solve(prob, {"Ks": Ks.reshape(n, n)}, n, opts, mode="mg")
    r["qoi"] = oqoi.mean_saturation(prob, {"Ks": Ks.reshape(n, n)}, r["p"]) if r["status"] == 0 else np.nan
    return r


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
