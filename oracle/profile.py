"""Laterally averaged charge density and electrostatic potential profile.

Written from the paper's potential-profile subsection (Eq. 16) and the
post-analysis paragraph of the appendix: the charge density rho(z) across
the cell, with the electrode charges as their Gaussian distributions, is
averaged over frames on a z-grid, and the 1D Poisson equation

    d^2 psi / dz^2 = -rho(z) / eps0

is solved with a matrix-based finite-difference method (the second
difference (psi_{k+1} - 2 psi_k + psi_{k-1}) / h^2 on the grid, inverted by
a linear solve).  Boundary conditions, per geometry:

* finite field: the potential rises by dpsi over one period,
  psi(Lz) - psi(0) = dpsi (a discontinuity across the cell boundary);
* doubled cell: continuity, psi(Lz) - psi(0) = 0;
* slab: no field in the empty space at the boundary (the corrected slab is
  isolated in z), i.e. the finite-difference equations with zero-flux ends.

The bulk potential, the mean of psi over a window of grid points in the
middle of the electrolyte, is subtracted.

Grid: n bins of width h = Lz/n, bin k = [k h, (k+1) h), values at the bin
centres.  Electrolyte point charges are counted in the bin holding their
wrapped z; an electrode atom's charge q_i contributes its Gaussian
(Eq. 2, marginal q_i eta/sqrt(pi) exp(-eta^2 (z - z_i)^2) along z)
integrated over each bin, periodic images included.  Densities are per
volume (e / nm^3): charge per bin divided by Lx Ly h.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import KE

EPS0 = 1.0 / (4.0 * math.pi * KE)   # e / (V nm)


def density(w, site_frames, elec_q_frames, n_bins):
    """Frame-averaged rho on the grid: site_frames (F, 3, n_site), elec_q_frames (F, n_elec)."""
    lz = w.box[2]
    h = lz / n_bins
    area = w.box[0] * w.box[1]
    edges = np.arange(n_bins + 1) * h
    charge = np.zeros(n_bins)
    nf = site_frames.shape[0]
    for f in range(nf):
        z = site_frames[f, 2] - lz * np.floor(site_frames[f, 2] / lz)
        k = np.minimum((z / h).astype(np.int64), n_bins - 1)
        np.add.at(charge, k, w.site_q)
    ze = w.elec_xyz[2] - lz * np.floor(w.elec_xyz[2] / lz)
    qbar = elec_q_frames.sum(axis=0)
    for img in (-1, 0, 1):
        c = ze + img * lz
        cdf = 0.5 * erf(w.eta * (edges[None, :] - c[:, None]))       # (n_elec, n_bins + 1)
        charge += qbar @ np.diff(cdf, axis=1)
    return charge / nf / (area * h)


def poisson_matrix(n_bins, h, geometry):
    """The second-difference matrix (1/h^2 units) with the geometry's ends."""
    D = np.zeros((n_bins, n_bins))
    for k in range(n_bins):
        D[k, k] = -2.0
        if k > 0:
            D[k, k - 1] = 1.0
        if k < n_bins - 1:
            D[k, k + 1] = 1.0
    if geometry == "slab":
        D[0, 0] = -1.0              # ghost point psi_{-1} = psi_0 (zero flux)
        D[-1, -1] = -1.0            # ghost point psi_n = psi_{n-1}
    else:
        D[0, -1] = 1.0              # periodic neighbours across the boundary
        D[-1, 0] = 1.0
    return D / (h * h)


def potential(rho, box, geometry, dv, bulk):
    """psi on the grid from rho by the finite-difference solve; bulk = (z_lo, z_hi)
    window whose mean potential is set to zero."""
    n = rho.size
    h = box[2] / n
    D = poisson_matrix(n, h, geometry)
    rhs = -rho / EPS0
    if geometry == "ff":
        # psi_{-1} = psi_{n-1} - dv and psi_n = psi_0 + dv (rise of dv over a period)
        rhs = rhs.copy()
        rhs[0] += dv / (h * h)
        rhs[-1] -= dv / (h * h)
    # the matrix is singular (constants); fix the constant with a multiplier row
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = D
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    sol = np.linalg.solve(M, np.concatenate([rhs, [0.0]]))
    psi = sol[:n]
    zc = (np.arange(n) + 0.5) * h
    sel = (zc >= bulk[0]) & (zc < bulk[1])
    return psi - psi[sel].mean()
