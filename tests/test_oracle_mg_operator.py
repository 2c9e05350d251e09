"""Pin of the oracle's multigrid cycle (Section 4.2) by its error-propagation operator.

A cycle with a zero right-hand side maps the initial error e to E e.  E is built here
from matrices alone, independently of the oracle's cycle code:
  * red-black Gauss-Seidel: a half-sweep of one colour is I - M D^-1 A (M selects the
    colour's cells, which the five-point operator does not couple to one another), red
    ((i + j) even) first; lexicographic Gauss-Seidel is I - (D + L)^-1 A with L the strictly
    lower part in the order x fastest, bottom row first;
  * transfers: P the piecewise-constant injection (a Kronecker product of 1-D injections),
    R = P^T / 4 (eq. transfer);
  * recursion: E = S^nu2 (I - P (I - E_c^gamma) A_c^-1 R A) S^nu1 with E_c the next level's
    operator and E = 0 on the exactly solved coarsest level.
The constant-coefficient operators come from Kronecker products (Neumann sides, half-cell
Dirichlet top and bottom), the heterogeneous ones from the oracle's coarsening and
assembly, which are pinned elsewhere (hand-worked coarsening, direct discretisation,
symmetric M-matrix).  The oracle's cycle must reproduce E column by column, and its
measured asymptotic contraction must be E's spectral radius: the convergence factor that
sets the Picard and cycle counts follows from the iteration matrix.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fv, kl, mg


def kron_operator(n, k0, cdt0):
    h = 1.0 / n
    Tx = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    Tx[0, 0] = Tx[n - 1, n - 1] = 1.0
    Tz = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    Tz[0, 0] = Tz[n - 1, n - 1] = 3.0
    I = sp.identity(n)
    return ((k0 / h ** 2) * (sp.kron(I, Tx) + sp.kron(Tz, I)) + cdt0 * sp.identity(n * n)).toarray()


def injection(nc):
    P1 = np.zeros((2 * nc, nc))
    for I in range(nc):
        P1[2 * I, I] = P1[2 * I + 1, I] = 1.0
    return np.kron(P1, P1)


def smoother(A, n, kind):
    N = n * n
    D = np.diag(A)
    if kind == "rb":
        jj, ii = np.divmod(np.arange(N), n)
        red = ((ii + jj) % 2 == 0).astype(float)
        S_red = np.eye(N) - (red / D)[:, None] * A
        S_black = np.eye(N) - ((1.0 - red) / D)[:, None] * A
        return S_black @ S_red
    DL = np.tril(A)
    return np.eye(N) - np.linalg.solve(DL, A)


def error_operator(As, ns, gamma, nu1, nu2, kind):
    """E of a cycle on level 0 of the hierarchy As (dense operators, finest first)."""
    E = np.zeros_like(As[-1])
    for l in range(len(As) - 2, -1, -1):
        A, Ac, n = As[l], As[l + 1], ns[l]
        P = injection(n // 2)
        R = P.T / 4.0
        Ec = np.linalg.matrix_power(E, gamma)
        cgc = np.eye(n * n) - P @ (np.eye(Ac.shape[0]) - Ec) @ np.linalg.solve(Ac, R @ A)
        S = smoother(A, n, kind)
        E = np.linalg.matrix_power(S, nu2) @ cgc @ np.linalg.matrix_power(S, nu1)
    return E


def oracle_operator(levels, gamma, nu1, nu2, kind):
    n = levels[0].n
    cols = []
    f = np.zeros((n, n))
    for k in range(n * n):
        u = np.zeros(n * n)
        u[k] = 1.0
        out = mg.cycle(levels, f, u.reshape(n, n).copy(), gamma=gamma, nu1=nu1, nu2=nu2, smoother=kind)
        cols.append(out.ravel())
    return np.array(cols).T


def constant_hierarchy(n, k0, cdt0):
    kx, kz = fv.face_conductivities(np.full((n, n), k0))
    levels = mg.hierarchy(kx, kz, np.full((n, n), cdt0), 4)
    ns = [lev.n for lev in levels]
    return levels, [kron_operator(m, k0, cdt0) for m in ns], ns


@pytest.mark.parametrize("n,gamma,nu,kind", [(8, 1, (2, 2), "rb"), (16, 1, (2, 2), "rb"), (16, 2, (2, 2), "rb"),
                                             (16, 1, (1, 3), "rb"), (16, 1, (2, 2), "lex")])
def test_constant_coefficient_cycle_is_its_iteration_matrix(n, gamma, nu, kind):
    levels, As, ns = constant_hierarchy(n, 0.8, 2.5)
    E = error_operator(As, ns, gamma, nu[0], nu[1], kind)
    Eo = oracle_operator(levels, gamma, nu[0], nu[1], kind)
    assert np.max(np.abs(Eo - E)) <= 1e-12 * np.max(np.abs(E))


def test_heterogeneous_cycle_is_its_iteration_matrix(kl_basis_small):
    lam, B = kl_basis_small
    n = 16
    xi = W.xi_draws(7, 0, [3], 1, B[n].shape[0])[0, 0]
    Kc = kl.lognormal(kl.gaussian_field(xi, B[n]), scale=1.5).reshape(n, n)
    kx, kz = fv.face_conductivities(Kc)
    cdt = W.uniform_array([9, n], (n, n), 0.0, 2.0)
    levels = mg.hierarchy(kx, kz, cdt, 4)
    As = [fv.assemble(lev.st).toarray() for lev in levels]
    ns = [lev.n for lev in levels]
    for gamma in (1, 2):
        E = error_operator(As, ns, gamma, 2, 2, "rb")
        Eo = oracle_operator(levels, gamma, 2, 2, "rb")
        assert np.max(np.abs(Eo - E)) <= 1e-12 * np.max(np.abs(E)), gamma


def test_measured_contraction_is_the_spectral_radius():
    """Repeated V(2,2) cycles on a zero right-hand side contract a generic error by the
    spectral radius of E per cycle, asymptotically."""
    n = 32
    levels, As, ns = constant_hierarchy(n, 1.0, 0.0)
    rho = np.max(np.abs(np.linalg.eigvals(error_operator(As, ns, 1, 2, 2, "rb"))))
    assert 0.0 < rho < 0.5
    u = W.normal_array([11, n], (n, n))
    f = np.zeros((n, n))
    ratios = []
    for _ in range(40):
        before = np.linalg.norm(u)
        u = mg.cycle(levels, f, u)
        ratios.append(np.linalg.norm(u) / before)
        u /= np.linalg.norm(u)  # keep the iterate away from underflow
    assert abs(np.mean(ratios[-5:]) - rho) <= 1e-3 * rho
