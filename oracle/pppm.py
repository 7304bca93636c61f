"""Particle-particle particle-mesh (PPPM) sums with the same Ewald splitting.

The paper evaluates the long-range electrostatics with Hockney-Eastwood
PPPM (appendix, force-field paragraph; the b vector of Eq. (3) is the
"main computational burden" of each charge update, Sec. II.A).  The paper
does not print the PPPM details; this module fixes them as:

* charge assignment: cardinal B-spline of order P (P = 5 in all workloads),
  centred on the particle, on a Kx x Ky x Kz mesh with spacing h = L/K;
* influence function: the Hockney-Eastwood optimal function for ik
  differentiation with aliases m in each axis such that |n + mK| <= 2.5 K
  (5 aliases, 6 at the Nyquist index so the set is symmetric);
* potential: phi_M = (1/V) sum_k G(k) rho_hat(k) e^{ik.x_m}, interpolated
  back with the same B-spline weights;
* field: ik differentiation, E_M = -(1/V) sum_k i D(k) G rho_hat e^{ik.x_m}
  with D(k) = k except a zero component at the Nyquist index.

The short-range parts are the real-space sums of ``oracle.ewald`` with
cutoff rcut.
"""

from __future__ import annotations

import math

import numpy as np

from . import KE
from . import ewald


def bspline(order, x):
    """Cardinal B-spline M_order(x), supported on [0, order].

    Cox-de Boor recursion: M_1 = indicator of [0, 1),
    M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1).
    """
    x = np.asarray(x, dtype=np.float64)
    if order == 1:
        return ((x >= 0.0) & (x < 1.0)).astype(np.float64)
    return (x * bspline(order - 1, x) + (order - x) * bspline(order - 1, x - 1.0)) / (order - 1)


def assignment(xyz, box, mesh, order):
    """Mesh points and weights of every particle along each axis.

    The particle at scaled coordinate u = x/h (x wrapped into [0, L)) is
    spread with the centred spline W(t) = M_P(t + P/2) over the P mesh
    points m = floor(u - P/2) + 1, ..., floor(u - P/2) + P, weight W(u - m).
    Returns first[3, n] (unwrapped first index) and w[3, n, P].
    """
    box = np.asarray(box, dtype=np.float64)
    n = xyz.shape[1]
    first = np.empty((3, n), dtype=np.int64)
    w = np.empty((3, n, order))
    for d in range(3):
        x = xyz[d] - box[d] * np.floor(xyz[d] / box[d])
        u = x / (box[d] / mesh[d])
        m0 = np.floor(u - order / 2.0).astype(np.int64) + 1
        first[d] = m0
        for t in range(order):
            w[d, :, t] = bspline(order, u - (m0 + t) + order / 2.0)
    return first, w


def spread(xyz, q, box, mesh, order):
    """rho_M[mx, my, mz] = sum_j q_j W(x_j - x_m) (charge per mesh point)."""
    rho = np.zeros(mesh)
    first, w = assignment(xyz, box, mesh, order)
    for j in range(xyz.shape[1]):
        ix = (first[0, j] + np.arange(order)) % mesh[0]
        iy = (first[1, j] + np.arange(order)) % mesh[1]
        iz = (first[2, j] + np.arange(order)) % mesh[2]
        block = q[j] * w[0, j][:, None, None] * w[1, j][None, :, None] * w[2, j][None, None, :]
        rho[np.ix_(ix, iy, iz)] += block
    return rho


def interpolate(xyz, field, box, order):
    """Value of a mesh field at each particle: sum_m W(x_j - x_m) field[m]."""
    mesh = field.shape
    first, w = assignment(xyz, box, mesh, order)
    out = np.empty(xyz.shape[1])
    for j in range(xyz.shape[1]):
        ix = (first[0, j] + np.arange(order)) % mesh[0]
        iy = (first[1, j] + np.arange(order)) % mesh[1]
        iz = (first[2, j] + np.arange(order)) % mesh[2]
        block = w[0, j][:, None, None] * w[1, j][None, :, None] * w[2, j][None, None, :]
        out[j] = np.sum(block * field[np.ix_(ix, iy, iz)])
    return out


def mesh_wavevectors(box, mesh):
    """Integer mode numbers n_d (numpy FFT order) and k_d = 2 pi n_d / L_d per axis."""
    ns = [np.fft.fftfreq(K, d=1.0 / K).round().astype(np.int64) for K in mesh]
    ks = [2 * math.pi * n / L for n, L in zip(ns, box)]
    return ns, ks


def influence(box, mesh, order, alpha, nalias=2):
    """Hockney-Eastwood optimal influence function for ik differentiation.

    G(k) = sum_m U^2(k_m) (k . k_m) R(k_m) / ( |k|^2 [sum_m U^2(k_m)]^2 ),
    k_m = k + 2 pi m / h, U(k) = prod_d [sin(k_d h_d/2)/(k_d h_d/2)]^P,
    R(k) = 4 pi exp(-k^2 / 4 alpha^2) / k^2, G(0) = 0.  The alias set in
    axis d is every m_d with |n_d + m_d K_d| <= (nalias + 1/2) K_d.
    """
    box = np.asarray(box, dtype=np.float64)
    ns, ks = mesh_wavevectors(box, mesh)
    h = box / np.asarray(mesh)
    # per axis, alias wavevectors and U^2 factors on a padded range of m,
    # with U^2 = 0 for the m outside the alias set
    mrange = np.arange(-nalias - 1, nalias + 2)
    ka, u2 = [], []
    for d in range(3):
        K = mesh[d]
        nm = ns[d][:, None] + mrange[None, :] * K            # (K, 2 nalias + 3)
        kk = 2 * math.pi * nm / box[d]
        arg = kk * h[d] / 2.0
        safe = np.where(arg == 0.0, 1.0, arg)
        sinc = np.where(arg == 0.0, 1.0, np.sin(safe) / safe)
        inside = np.abs(nm) <= (nalias + 0.5) * K
        ka.append(kk)
        u2.append(np.where(inside, sinc ** (2 * order), 0.0))
    kx, ky, kz = np.meshgrid(ks[0], ks[1], ks[2], indexing="ij")
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    num = np.zeros(mesh)
    den = np.zeros(mesh)
    nm_ = len(mrange)
    for a in range(nm_):
        for b in range(nm_):
            for c in range(nm_):
                KX = ka[0][:, a][:, None, None]
                KY = ka[1][:, b][None, :, None]
                KZ = ka[2][:, c][None, None, :]
                U2 = u2[0][:, a][:, None, None] * u2[1][:, b][None, :, None] * u2[2][:, c][None, None, :]
                km2 = KX ** 2 + KY ** 2 + KZ ** 2
                km2s = np.where(km2 == 0.0, 1.0, km2)
                R = np.where(km2 == 0.0, 0.0, 4 * math.pi * np.exp(-km2 / (4 * alpha * alpha)) / km2s)
                num += U2 * (kx * KX + ky * KY + kz * KZ) * R
                den += U2
    G = np.zeros(mesh)
    nz = k2 > 0
    G[nz] = num[nz] / (k2[nz] * den[nz] ** 2)
    return G


def nyquist_free(ns_d, K):
    """1 where the mode is not the Nyquist index of an even-length axis, else 0."""
    if K % 2 == 0:
        return (ns_d != -(K // 2)).astype(np.float64)
    return np.ones_like(ns_d, dtype=np.float64)


def mesh_potential(rho, G, box):
    """phi_M = (1/V) sum_k G(k) rho_hat(k) exp(i k.x_m), rho_hat = DFT of rho_M (no k_e)."""
    n = rho.size
    vol = float(np.prod(box))
    return np.real(np.fft.ifftn(G * np.fft.fftn(rho))) * n / vol


def mesh_field(rho, G, box):
    """E_M,d = -(1/V) sum_k i D_d(k) G rho_hat exp(i k.x_m) (no k_e); (3, Kx, Ky, Kz)."""
    mesh = rho.shape
    n = rho.size
    vol = float(np.prod(box))
    ns, ks = mesh_wavevectors(box, mesh)
    rho_hat = np.fft.fftn(rho)
    out = np.empty((3,) + mesh)
    for d in range(3):
        D = ks[d] * nyquist_free(ns[d], mesh[d])
        shape = [1, 1, 1]
        shape[d] = mesh[d]
        Dd = D.reshape(shape)
        out[d] = np.real(np.fft.ifftn(-1j * Dd * G * rho_hat)) * n / vol
    return out


def b_vector(elec_xyz, site_xyz, site_q, box, eta, alpha, rcut, mesh, order, G=None):
    """b of Eq. (3) with the reciprocal part from the mesh.

    b_i = -[ k_e sum_j Q_j sum_n g1 (r < rcut) + k_e phi_M interpolated at r_i ].
    """
    box = np.asarray(box, dtype=np.float64)
    if G is None:
        G = influence(box, mesh, order, alpha)
    real = ewald.electrolyte_potential_realspace(elec_xyz, site_xyz, site_q, box, eta, alpha, rcut)
    rho = spread(site_xyz, site_q, box, mesh, order)
    phi = mesh_potential(rho, G, box)
    recip = KE * interpolate(elec_xyz, phi, box, order)
    return -(real + recip)


def electrolyte_energy(site_xyz, site_q, box, alpha, rcut, mesh, order, G=None):
    """U_elyt with the mesh energy 1/2 sum_m rho_M phi_M in place of the k-sum."""
    box = np.asarray(box, dtype=np.float64)
    if G is None:
        G = influence(box, mesh, order, alpha)
    m = ewald.realspace_matrix(site_xyz, site_xyz, box, rcut, lambda r: ewald.g0(r, alpha),
                               exclude_self=True)
    real = 0.5 * site_q @ m @ site_q
    rho = spread(site_xyz, site_q, box, mesh, order)
    recip = 0.5 * np.sum(rho * mesh_potential(rho, G, box))
    self_e = alpha / math.sqrt(math.pi) * np.sum(site_q ** 2)
    return KE * (real + recip - self_e)


def coulomb_forces(site_xyz, site_q, elec_xyz, elec_q, box, eta, alpha, rcut, mesh, order, G=None):
    """Coulomb force on the electrolyte sites, reciprocal part by ik-PPPM over all charges."""
    box = np.asarray(box, dtype=np.float64)
    if G is None:
        G = influence(box, mesh, order, alpha)
    f_ll = ewald.realspace_vector_field(site_xyz, site_xyz, site_q, box, rcut,
                                        lambda r: ewald.g0_force(r, alpha), exclude_self=True)
    f_le = ewald.realspace_vector_field(site_xyz, elec_xyz, elec_q, box, rcut,
                                        lambda r: ewald.g1_force(r, alpha, eta))
    rho = spread(site_xyz, site_q, box, mesh, order) + spread(elec_xyz, elec_q, box, mesh, order)
    E = mesh_field(rho, G, box)
    fk = np.stack([interpolate(site_xyz, E[d], box, order) for d in range(3)])
    return KE * site_q[None, :] * (f_ll + f_le + fk)
