"""Exact Ewald sums for point electrolyte charges and Gaussian electrode charges.

Follows the energy of the paper's Eq. (1) with the electrode densities of
Eq. (2) and the quadratic form of Eq. (3).  The Coulomb interaction of

    two point charges          1/r
    a point and a Gaussian     erf(eta r)/r
    two Gaussians              erf(eta r / sqrt 2)/r

is split with the usual Ewald parameter alpha into a short-range part that
is summed over periodic images in real space,

    g0(r) = erfc(alpha r)/r
    g1(r) = [erfc(alpha r) - erfc(eta r)]/r
    g2(r) = [erfc(alpha r) - erfc(eta r / sqrt 2)]/r,

and the long-range erf(alpha r)/r part, which is summed in reciprocal space
with weight w(k) = (4 pi / V) exp(-k^2 / 4 alpha^2) / k^2 over k != 0
(conducting "tinfoil" boundary).  Fully periodic boundaries throughout, as
in the paper's finite-field and doubled-cell geometries (Sec. II.B).

All lengths nm, charges e, potentials V, energies eV.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import KE

SQRT_PI = math.sqrt(math.pi)


# --------------------------------------------------------------------------
# pair kernels
# --------------------------------------------------------------------------

def g0(r, alpha):
    """Short-range point-point kernel erfc(alpha r)/r."""
    return erfc(alpha * r) / r


def g1(r, alpha, eta):
    """Short-range point-Gaussian kernel [erfc(alpha r) - erfc(eta r)]/r."""
    return (erfc(alpha * r) - erfc(eta * r)) / r


def g2(r, alpha, eta):
    """Short-range Gaussian-Gaussian kernel [erfc(alpha r) - erfc(eta r/sqrt2)]/r."""
    return (erfc(alpha * r) - erfc(eta * r / math.sqrt(2.0))) / r


def g0_force(r, alpha):
    """-d g0/dr."""
    return erfc(alpha * r) / r ** 2 + 2.0 * alpha / SQRT_PI * np.exp(-(alpha * r) ** 2) / r


def g1_force(r, alpha, eta):
    """-d g1/dr."""
    return ((erfc(alpha * r) - erfc(eta * r)) / r ** 2
            + 2.0 / SQRT_PI * (alpha * np.exp(-(alpha * r) ** 2)
                               - eta * np.exp(-(eta * r) ** 2)) / r)


# --------------------------------------------------------------------------
# real-space image sums
# --------------------------------------------------------------------------

def image_shifts(box, rcut):
    """All lattice vectors n*L that can bring a minimum-image pair within rcut.

    After the minimum-image reduction each displacement component lies in
    [-L/2, L/2], so |d + n L| < rcut needs |n| <= floor(rcut/L + 1/2).
    """
    m = [int(math.floor(rcut / L + 0.5)) for L in box]
    shifts = [(a * box[0], b * box[1], c * box[2])
              for a in range(-m[0], m[0] + 1)
              for b in range(-m[1], m[1] + 1)
              for c in range(-m[2], m[2] + 1)]
    return np.array(shifts, dtype=np.float64)


def _min_image(d, box):
    return d - box[:, None, None] * np.round(d / box[:, None, None])


def realspace_matrix(xa, xb, box, rcut, kernel, exclude_self=False, chunk=256):
    """M[a, b] = sum over images n of kernel(|x_a - x_b + n L|), |.| < rcut.

    xa (3, na), xb (3, nb).  With exclude_self the n = 0 term of a == b is
    left out (xa and xb must then be the same set).
    """
    box = np.asarray(box, dtype=np.float64)
    na, nb = xa.shape[1], xb.shape[1]
    out = np.zeros((na, nb))
    shifts = image_shifts(box, rcut)
    for a0 in range(0, na, chunk):
        a1 = min(na, a0 + chunk)
        d0 = _min_image(xa[:, a0:a1, None] - xb[:, None, :], box)
        for s in shifts:
            d = d0 + s[:, None, None]
            r = np.sqrt(np.einsum("kab,kab->ab", d, d))
            mask = r < rcut
            if exclude_self and not np.any(s):
                idx = np.arange(a0, a1)
                mask[idx - a0, idx] = False
            rr = np.where(mask, r, 1.0)
            out[a0:a1] += np.where(mask, kernel(rr), 0.0)
    return out


def realspace_vector_field(xa, xb, qb, box, rcut, radial, exclude_self=False, chunk=256):
    """F[:, a] = sum_b q_b sum_n radial(r) * (x_a - x_b + n L)/r, r < rcut.

    radial(r) is -d(kernel)/dr, so F is the force on a unit charge at x_a.
    """
    box = np.asarray(box, dtype=np.float64)
    na = xa.shape[1]
    out = np.zeros((3, na))
    shifts = image_shifts(box, rcut)
    for a0 in range(0, na, chunk):
        a1 = min(na, a0 + chunk)
        d0 = _min_image(xa[:, a0:a1, None] - xb[:, None, :], box)
        for s in shifts:
            d = d0 + s[:, None, None]
            r = np.sqrt(np.einsum("kab,kab->ab", d, d))
            mask = r < rcut
            if exclude_self and not np.any(s):
                idx = np.arange(a0, a1)
                mask[idx - a0, idx] = False
            rr = np.where(mask, r, 1.0)
            f = np.where(mask, radial(rr) / rr, 0.0) * qb[None, :]
            out[:, a0:a1] += np.einsum("kab,ab->ka", d, f)
    return out


# --------------------------------------------------------------------------
# reciprocal space
# --------------------------------------------------------------------------

def kvectors(box, kcut):
    """All k = 2 pi (n1/Lx, n2/Ly, n3/Lz) with 0 < |k| <= kcut (both k and -k)."""
    box = np.asarray(box, dtype=np.float64)
    nmax = [int(math.floor(kcut * L / (2 * math.pi))) for L in box]
    n = np.stack(np.meshgrid(*[np.arange(-m, m + 1) for m in nmax], indexing="ij"), -1).reshape(-1, 3)
    k = 2 * math.pi * n / box[None, :]
    k2 = np.sum(k * k, axis=1)
    keep = (k2 > 0) & (k2 <= kcut * kcut)
    return k[keep]


def kweight(k, box, alpha):
    """w(k) = (4 pi / V) exp(-k^2/(4 alpha^2)) / k^2."""
    vol = float(np.prod(box))
    k2 = np.sum(k * k, axis=1)
    return 4 * math.pi / vol * np.exp(-k2 / (4 * alpha * alpha)) / k2


def structure_factor(k, xyz, q, chunk=4096):
    """rho_hat(k) = sum_j q_j exp(i k . R_j)."""
    out = np.empty(k.shape[0], dtype=np.complex128)
    for k0 in range(0, k.shape[0], chunk):
        ph = k[k0:k0 + chunk] @ xyz
        out[k0:k0 + chunk] = np.exp(1j * ph) @ q
    return out


# --------------------------------------------------------------------------
# the pieces of Eq. (3)
# --------------------------------------------------------------------------

def elastance(elec_xyz, box, eta, alpha, rcut, kcut):
    """Electrode-electrode matrix A of Eq. (3), in V/e.

    A_ii' = k_e [ sum_n* g2(|r_i - r_i' + nL|)
                  + sum_k w(k) cos(k.(r_i - r_i'))
                  + delta_ii' (sqrt2 eta - 2 alpha)/sqrt(pi) ],
    the starred sum leaving out n = 0 for i = i'.  The last term is the
    Gaussian self-interaction sqrt2 eta/sqrt(pi) minus the alpha-Gaussian
    self-term included in the k-space sum.
    """
    box = np.asarray(box, dtype=np.float64)
    real = realspace_matrix(elec_xyz, elec_xyz, box, rcut, lambda r: g2(r, alpha, eta),
                            exclude_self=True)
    k = kvectors(box, kcut)
    w = kweight(k, box, alpha)
    ph = k @ elec_xyz                       # (Nk, Ne)
    # sum_k w cos(k.(r_i - r_j)) written as the product of cos/sin factors
    c = np.sqrt(w)[:, None] * np.cos(ph)
    s = np.sqrt(w)[:, None] * np.sin(ph)
    recip = c.T @ c + s.T @ s
    self_term = (math.sqrt(2.0) * eta - 2.0 * alpha) / SQRT_PI
    return KE * (real + recip + self_term * np.eye(elec_xyz.shape[1]))


def electrolyte_potential_realspace(elec_xyz, site_xyz, site_q, box, eta, alpha, rcut):
    """k_e sum_j Q_j sum_n g1(|r_i - R_j + n L|): short-range part of -b."""
    m = realspace_matrix(elec_xyz, site_xyz, box, rcut, lambda r: g1(r, alpha, eta))
    return KE * (m @ site_q)


def b_vector(elec_xyz, site_xyz, site_q, box, eta, alpha, rcut, kcut):
    """Electrolyte vector b of Eq. (3): b_i = -(potential of the electrolyte at the Gaussian i).

    b_i = -k_e [ sum_j Q_j sum_n g1(|r_i - R_j + nL|)
                 + sum_k w(k) Re(exp(-i k.r_i) rho_hat(k)) ].
    """
    box = np.asarray(box, dtype=np.float64)
    real = electrolyte_potential_realspace(elec_xyz, site_xyz, site_q, box, eta, alpha, rcut)
    k = kvectors(box, kcut)
    w = kweight(k, box, alpha)
    rho = structure_factor(k, site_xyz, site_q)
    recip = np.empty(elec_xyz.shape[1])
    for i0 in range(0, elec_xyz.shape[1], 512):
        ph = k @ elec_xyz[:, i0:i0 + 512]
        recip[i0:i0 + 512] = np.real(np.exp(-1j * ph) * rho[:, None]).T @ w
    return -(real + KE * recip)


def electrolyte_energy(site_xyz, site_q, box, alpha, rcut, kcut):
    """U_elyt of Eq. (3): point-point Ewald energy of the electrolyte.

    U = k_e [ 1/2 sum'_{j,j',n} Q_j Q_j' g0 + 1/2 sum_k w |rho_hat|^2
              - alpha/sqrt(pi) sum_j Q_j^2 ].
    """
    box = np.asarray(box, dtype=np.float64)
    m = realspace_matrix(site_xyz, site_xyz, box, rcut, lambda r: g0(r, alpha), exclude_self=True)
    real = 0.5 * site_q @ m @ site_q
    k = kvectors(box, kcut)
    w = kweight(k, box, alpha)
    rho = structure_factor(k, site_xyz, site_q)
    recip = 0.5 * np.sum(w * np.abs(rho) ** 2)
    self_e = alpha / SQRT_PI * np.sum(site_q ** 2)
    return KE * (real + recip - self_e)


def coulomb_forces(site_xyz, site_q, elec_xyz, elec_q, box, eta, alpha, rcut, kcut):
    """Coulomb force on every electrolyte site at fixed electrode charges.

    F_j = -dU/dR_j of U_elyt - q.b (electrodes fixed): the real-space g0
    pairs with other sites, the g1 pairs with Gaussian electrode charges and
    the reciprocal sum over all charges,
        F_j^k = -k_e Q_j sum_k w(k) k Im(exp(-i k.R_j) rho_all(k)).
    Returns (3, n_site) in eV/nm.
    """
    box = np.asarray(box, dtype=np.float64)
    f_ll = realspace_vector_field(site_xyz, site_xyz, site_q, box, rcut,
                                  lambda r: g0_force(r, alpha), exclude_self=True)
    f_le = realspace_vector_field(site_xyz, elec_xyz, elec_q, box, rcut,
                                  lambda r: g1_force(r, alpha, eta))
    k = kvectors(box, kcut)
    w = kweight(k, box, alpha)
    rho = structure_factor(k, site_xyz, site_q) + structure_factor(k, elec_xyz, elec_q)
    fk = np.empty((3, site_xyz.shape[1]))
    for j0 in range(0, site_xyz.shape[1], 512):
        ph = k @ site_xyz[:, j0:j0 + 512]
        im = np.imag(np.exp(-1j * ph) * rho[:, None])   # (Nk, nj)
        fk[:, j0:j0 + 512] = -(k * w[:, None]).T @ im
    return KE * site_q[None, :] * (f_ll + f_le + fk)
