"""Cell-centred finite volumes on the unit square (oracle, FP64).

Grid (Section 4.2 eq. Grid_fine): n x n cells of width h = 1/n, centres
x_i = (i + 1/2) h, z_j = (j + 1/2) h (zero-based), arrays indexed [j, i] with
j = 0 the bottom row and z pointing up.

Darcy flux q = -K (grad p + e_z) (Section 2 eq. darcy); the mixed form
(eq. mixedForm) backward-Euler discretised (Section 4.1 eq. Mixed_based) gives,
per cell, the Picard right-hand side

    f~_c = (net inflow through the faces of c) / h^2  -  (theta_c - theta_c^old) / dt

with face conductivity equal to the harmonic mean of the two adjacent cell
conductivities (Section 4.2, stencil eq. five_stencil).  The paper leaves the
boundary stencil to be "modified appropriately"; the reading used here is

  * top (z = 1) and bottom (z = 0): Dirichlet, the face conductivity is that of
    the adjacent cell and the pressure difference spans h/2 (mirror ghost cell);
  * sides (x = 0, 1): no flux, the face carries nothing;
  * the gravity term uses the same face conductivity as the diffusion term
    (conservative flux form).

Face arrays: kx[j, i] for i = 0..n is the x-face left of cell i (kx[:, 0] and
kx[:, n] are the no-flux sides and stay 0); kz[j, i] for j = 0..n is the z-face
below cell row j (kz[0] and kz[n] are the Dirichlet bottom and top faces).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def harmonic_mean(a, b):
    """2ab/(a+b), the face value of eq. five_stencil (0 when both vanish)."""
    s = a + b
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(s > 0.0, 2.0 * a * b / np.where(s > 0.0, s, 1.0), 0.0)


def face_conductivities(Kc):
    """Harmonic-mean face conductivities of a cell field Kc[j, i]; Dirichlet faces take the cell value."""
    n = Kc.shape[0]
    kx = np.zeros((n, n + 1))
    kz = np.zeros((n + 1, n))
    kx[:, 1:n] = harmonic_mean(Kc[:, :-1], Kc[:, 1:])
    kz[1:n, :] = harmonic_mean(Kc[:-1, :], Kc[1:, :])
    kz[0, :] = Kc[0, :]
    kz[n, :] = Kc[n - 1, :]
    return kx, kz


def net_inflow(p, kx, kz, h, g_bottom, g_top):
    """Sum over the faces of each cell of the inflow K_f((p_nb - p_c)/d_f + g_f) * h, divided by h^2.

    g_f = -1 through a bottom face and +1 through a top face (gravity, z up), 0 on x-faces;
    d_f = h between cells and h/2 from a cell centre to a Dirichlet face.
    """
    n = p.shape[0]
    q = np.zeros_like(p)
    # x-faces between cells i-1 and i: inflow into i is kx (p_{i-1} - p_i)/h per unit length
    fx = kx[:, 1:n] * (p[:, :-1] - p[:, 1:]) / h
    q[:, 1:] += fx
    q[:, :-1] -= fx
    # z-faces between rows j-1 and j: upward flux K((p_{j-1} - p_j)/h - 1)
    fz = kz[1:n, :] * ((p[:-1, :] - p[1:, :]) / h - 1.0)
    q[1:, :] += fz
    q[:-1, :] -= fz
    # Dirichlet bottom face: upward inflow into row 0
    q[0, :] += kz[0, :] * ((g_bottom - p[0, :]) / (0.5 * h) - 1.0)
    # Dirichlet top face: downward inflow into row n-1
    q[n - 1, :] += kz[n, :] * ((g_top - p[n - 1, :]) / (0.5 * h) + 1.0)
    return q / h


def boundary_inflow_total(p, kz, h, g_bottom, g_top):
    """Net volumetric inflow through the Dirichlet boundary per unit time (for the mass-balance pin)."""
    n = p.shape[0]
    bot = kz[0, :] * ((g_bottom - p[0, :]) / (0.5 * h) - 1.0)
    top = kz[n, :] * ((g_top - p[n - 1, :]) / (0.5 * h) + 1.0)
    return h * (np.sum(bot) + np.sum(top))


def picard_rhs(p, theta, theta_old, kx, kz, h, dt, g_bottom, g_top):
    """Right-hand side f~ of the correction equation (Section 4.1 eq. Mixed_based_3, f = 0)."""
    return net_inflow(p, kx, kz, h, g_bottom, g_top) - (theta - theta_old) / dt


def stencil(kx, kz, cdt, H):
    """Five-point stencil (w, e, s, n, c) of eq. five_stencil on mesh H for the correction dp.

    w, e, s, n multiply the neighbouring unknowns; a Dirichlet face (homogeneous
    for dp, Section 4.2 eq. diffusion_problem) has no neighbour and adds 2K/H^2 to
    the centre; no-flux faces add nothing.  cdt = C/dt per cell.
    """
    nn = cdt.shape[0]
    H2 = H * H
    w = -kx[:, 0:nn] / H2          # kx[:, 0] = 0: no-flux left side
    e = -kx[:, 1:nn + 1] / H2      # kx[:, nn] = 0: no-flux right side
    s = -kz[0:nn, :] / H2
    n_ = -kz[1:nn + 1, :] / H2
    s[0, :] = 0.0                  # bottom row: Dirichlet face, no neighbour
    n_[nn - 1, :] = 0.0            # top row: Dirichlet face, no neighbour
    c = -(w + e + s + n_) + cdt
    c[0, :] += 2.0 * kz[0, :] / H2        # mirror-ghost weight of the bottom Dirichlet face
    c[nn - 1, :] += 2.0 * kz[nn, :] / H2  # mirror-ghost weight of the top Dirichlet face
    return w, e, s, n_, c


def apply_stencil(st, u):
    """A u for a stencil tuple (w, e, s, n, c); neighbours outside the domain count as 0."""
    w, e, s, n_, c = st
    r = c * u
    r[:, 1:] += w[:, 1:] * u[:, :-1]
    r[:, :-1] += e[:, :-1] * u[:, 1:]
    r[1:, :] += s[1:, :] * u[:-1, :]
    r[:-1, :] += n_[:-1, :] * u[1:, :]
    return r


def assemble(st):
    """Sparse matrix of a stencil tuple with unknown index c = j*n + i."""
    w, e, s, n_, c = st
    nn = c.shape[0]
    N = nn * nn
    idx = np.arange(N).reshape(nn, nn)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [c.ravel()]
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(w[:, 1:].ravel())
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(e[:, :-1].ravel())
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(s[1:, :].ravel())
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(n_[:-1, :].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()
