"""Slab geometry: the electrodes and electrolyte periodic in x and y only.

The paper's reference setting (Faster Electrostatic Evaluation subsection,
Fig. 2b): z-periodicity is imposed on a box lengthened with empty space, and
the dipole-dipole interaction between the periodic copies is removed with a
charged-sheet correction (Yeh and Berkowitz).  For a neutral system with
total dipole moment M_z = sum_k q_k z_k in a box of volume V the corrected
energy is

    U = U_Ewald(3D) + k_e (2 pi / V) M_z^2,

which is exact for the laterally averaged (k_x = k_y = 0) part of the
electrostatics: the 3D-periodic one-dimensional Green's function differs
from the isolated one by -(z - z')^2 / 2 L_z, whose energy for a neutral
system is -(2 pi k_e / V) M_z^2.  The in-plane structure of the copies
interacts across the empty space only through terms that decay as
exp(-|G| gap).

In the constant-potential quadratic form (Eq. 3) the correction splits into
the three blocks:

    A  += k_e (4 pi / V) z z^T                 (electrode-electrode)
    b  -= k_e (4 pi / V) z M_elyt              (electrolyte-electrode)
    U_elyt += k_e (2 pi / V) M_elyt^2          (electrolyte-electrolyte)

with z the electrode heights and M_elyt = sum_j Q_j Z_j, and the force on
site j gains -k_e (4 pi / V) Q_j M_z along z, M_z = M_elyt + z.q.  The
electrode potentials are psibar e + dpsi d as in the doubled cell (one
electroneutrality constraint, no applied field).

Heights are taken in [0, Lz) of the lengthened box; the empty space must
contain the boundary z = 0 (the correction is only defined for a slab that
does not cross it).
"""

from __future__ import annotations

import math

import numpy as np

from . import KE


def heights(xyz, box):
    """z wrapped into [0, Lz)."""
    return xyz[2] - box[2] * np.floor(xyz[2] / box[2])


def kappa(box):
    """k_e 4 pi / V, the coefficient of the correction's second derivatives."""
    return KE * 4.0 * math.pi / float(np.prod(box))


def elastance_term(elec_xyz, box):
    z = heights(elec_xyz, box)
    return kappa(box) * np.outer(z, z)


def b_term(elec_xyz, site_xyz, site_q, box):
    return -kappa(box) * heights(elec_xyz, box) * (site_q @ heights(site_xyz, box))


def energy_term(site_xyz, site_q, box):
    m = site_q @ heights(site_xyz, box)
    return 0.5 * kappa(box) * m * m


def force_term(site_xyz, site_q, elec_xyz, elec_q, box):
    """(3, n_site) force of the correction on the sites at electrode charges elec_q."""
    m = site_q @ heights(site_xyz, box) + elec_q @ heights(elec_xyz, box)
    f = np.zeros((3, site_xyz.shape[1]))
    f[2] = -kappa(box) * site_q * m
    return f
