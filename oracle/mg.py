"""Cell-centred multigrid for the linearised Picard problem (oracle, FP64).

Section 4.2: uniform coarsening h -> 2h; coarse operators by direct
discretisation on the coarse grid, with coarse face conductivities upscaled as in
the figure on coefficient upscaling (fine faces: harmonic mean of cells; every
coarser face: arithmetic mean of the two finer faces it covers); piecewise
constant prolongation P and restriction R = P^T / 4 (eq. transfer).

Readings where the paper is silent:
  * coarse C/dt is the mean of the four fine values;
  * the coarsest grid (default 4 x 4) is solved exactly by dense Cholesky;
  * the smoother is Gauss-Seidel in red-black order (red = (i+j) even first),
    applied identically before and after the coarse correction; the paper's
    lexicographic order is available as an option;
  * the initial iterate on every level is zero.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import fv


class Level:
    """One grid of the hierarchy: face conductivities, C/dt and the resulting stencil."""

    def __init__(self, kx, kz, cdt):
        self.n = cdt.shape[0]
        self.H = 1.0 / self.n
        self.kx, self.kz, self.cdt = kx, kz, cdt
        self.st = fv.stencil(kx, kz, cdt, self.H)


def coarsen(level: Level) -> Level:
    """Arithmetic-mean face upscaling and mean-of-four C/dt (Section 4.2, upscaling figure)."""
    n = level.n
    nc = n // 2
    kx, kz, cdt = level.kx, level.kz, level.cdt
    # coarse x-face I of coarse row J covers fine x-faces 2I of fine rows 2J and 2J+1
    kxc = 0.5 * (kx[0::2, 0::2] + kx[1::2, 0::2])
    # coarse z-face J of coarse column I covers fine z-faces 2J of fine columns 2I and 2I+1
    kzc = 0.5 * (kz[0::2, 0::2] + kz[0::2, 1::2])
    cdtc = 0.25 * (cdt[0::2, 0::2] + cdt[0::2, 1::2] + cdt[1::2, 0::2] + cdt[1::2, 1::2])
    assert kxc.shape == (nc, nc + 1) and kzc.shape == (nc + 1, nc)
    return Level(kxc, kzc, cdtc)


def hierarchy(kx, kz, cdt, coarsest_n=4):
    levels = [Level(kx, kz, cdt)]
    while levels[-1].n > coarsest_n:
        levels.append(coarsen(levels[-1]))
    return levels


def restrict(r):
    """R = (1/4) [1 1; 1 1]: coarse value is the mean of the four fine values (eq. transfer)."""
    return 0.25 * (r[0::2, 0::2] + r[0::2, 1::2] + r[1::2, 0::2] + r[1::2, 1::2])


def prolong(uc):
    """P: piecewise constant injection of each coarse value into its four fine cells (eq. transfer)."""
    return np.repeat(np.repeat(uc, 2, axis=0), 2, axis=1)


def _neighbour_sum(st, u):
    w, e, s, n_, _ = st
    r = np.zeros_like(u)
    r[:, 1:] += w[:, 1:] * u[:, :-1]
    r[:, :-1] += e[:, :-1] * u[:, 1:]
    r[1:, :] += s[1:, :] * u[:-1, :]
    r[:-1, :] += n_[:-1, :] * u[1:, :]
    return r


def gs_red_black(st, u, f):
    """One red-black Gauss-Seidel sweep: red cells ((i+j) even), then black, each solving its own row."""
    nn = u.shape[0]
    jj, ii = np.indices((nn, nn))
    c = st[4]
    for colour in (0, 1):
        mask = ((ii + jj) % 2) == colour
        upd = (f - _neighbour_sum(st, u)) / c
        u[mask] = upd[mask]
    return u


def gs_lexicographic(st, u, f):
    """One lexicographic Gauss-Seidel sweep (the paper's smoother), x fastest, bottom row first."""
    w, e, s, n_, c = st
    nn = u.shape[0]
    for j in range(nn):
        for i in range(nn):
            acc = f[j, i]
            if i > 0:
                acc -= w[j, i] * u[j, i - 1]
            if i < nn - 1:
                acc -= e[j, i] * u[j, i + 1]
            if j > 0:
                acc -= s[j, i] * u[j - 1, i]
            if j < nn - 1:
                acc -= n_[j, i] * u[j + 1, i]
            u[j, i] = acc / c[j, i]
    return u


def coarsest_solve(level: Level, f):
    """Exact solve on the coarsest grid by dense Cholesky (the matrix is SPD)."""
    A = fv.assemble(level.st).toarray()
    cf = sla.cho_factor(A, lower=True)
    return sla.cho_solve(cf, f.ravel()).reshape(f.shape)


def cycle(levels, f, u=None, l=0, gamma=1, nu1=2, nu2=2, smoother="rb"):
    """One multigrid cycle on level l (gamma = 1: V-cycle, gamma = 2: W-cycle)."""
    lev = levels[l]
    if u is None:
        u = np.zeros_like(f)
    if l == len(levels) - 1:
        return coarsest_solve(lev, f)
    smooth = gs_red_black if smoother == "rb" else gs_lexicographic
    for _ in range(nu1):
        smooth(lev.st, u, f)
    r = f - fv.apply_stencil(lev.st, u)
    fc = restrict(r)
    uc = np.zeros_like(fc)
    for _ in range(gamma):
        uc = cycle(levels, fc, uc, l + 1, gamma, nu1, nu2, smoother)
    u += prolong(uc)
    for _ in range(nu2):
        smooth(lev.st, u, f)
    return u
