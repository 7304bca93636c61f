"""The electroneutral constant-potential solve, energy, forces and gradient.

Written from Sec. II.A-B of the paper:

* Eq. (4)   Psi = A q - b is the electrode potential vector;
* Eq. (5)   the target Psi = psibar e + dpsi d, d = +-1/2 per electrode;
* Eq. (7-9) electroneutrality e^T q = 0 fixes psibar and gives
            q* = O A^-1 (dpsi d + b), O = I - A^-1 e e^T / (e^T A^-1 e);
* Eq. (11)  finite field: q* = O A^-1 (-dpsi z / Lz + b);
* Eq. (12-15) doubled cell: a second constraint e1^T q = 0 adds
            O1 = I - O A^-1 e1 e1^T / (e1^T O A^-1 e1), q* = O1 O A^-1 (dpsi d + b).

Readings of the paper used here (all listed in the design notes):

* The applied field is E_z = -dpsi/Lz (Finite Field Method paragraph), so the
  field adds +dpsi z/Lz to the potential; Eq. (11) agrees, Eq. (10)'s sign
  does not and is taken as a misprint.
* With the electrolyte between the electrodes inside one cell, Eq. (11)
  puts dpsi across the electrolyte only if the lower electrode's z is taken
  one period up.  That is the same as using c = d - z/Lz with d = +1/2 on
  the upper electrode and wrapped z (the two differ by a multiple of e,
  which the projector removes).
* The charge solve is q* = S v with v = b + dpsi c, c = d (doubled cell) or
  d - z/Lz (finite field), and S = O A^-1 or O1 O A^-1.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from . import ewald, pppm, slab


def inverse_elastance(A):
    """A^-1 through a Cholesky factorisation (A is symmetric positive definite)."""
    c = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve(c, np.eye(A.shape[0]))


def projected_inverse(A, e1=None):
    """S = O A^-1 (Eq. 8-9), or O1 O A^-1 (Eq. 14-15) when e1 is given."""
    n = A.shape[0]
    e = np.ones(n)
    Ainv = inverse_elastance(A)
    O = np.eye(n) - np.outer(Ainv @ e, e) / (e @ Ainv @ e)
    S = O @ Ainv
    if e1 is not None:
        e1 = np.asarray(e1, dtype=np.float64)
        O1 = np.eye(n) - np.outer(S @ e1, e1) / (e1 @ S @ e1)
        S = O1 @ S
    return S


def drive_vector(w):
    """c with v = b + dpsi c: d for the doubled cell, d - z/Lz for the finite field.

    The finite-field form takes z wrapped into [0, Lz); it is Eq. (11) with
    the lower electrode's z taken one period up only if neither electrode
    crosses the cell boundary z = 0 (the ramp potential must be continuous
    inside each electrode), which is asserted here."""
    d = 0.5 * w.elec_side.astype(np.float64)
    if w.geometry in ("dc", "slab"):
        return d
    z = w.elec_xyz[2] - w.box[2] * np.floor(w.elec_xyz[2] / w.box[2])
    for side in (-1, 1):
        zs = z[w.elec_side == side]
        if zs.max() - zs.min() > 0.5 * w.box[2]:
            raise ValueError("a finite-field electrode crosses the cell boundary z = 0")
    return d - z / w.box[2]


def solve_charges(S, b, dv, c):
    """q* = S (b + dpsi c)."""
    return S @ (b + dv * c)


def sub_cell_vector(w):
    """e1: 1 on the electrode atoms of the first sub-cell (doubled cell only)."""
    if w.geometry != "dc":
        return None
    return w.elec_sub.astype(np.float64)


# --------------------------------------------------------------------------
# assembled evaluation for a workload
# --------------------------------------------------------------------------

def elastance(w):
    """A for the workload's electrodes with its converged Ewald parameters
    (plus the slab correction's z z^T block in slab geometry)."""
    A = ewald.elastance(w.elec_xyz, w.box, w.eta, w.alpha_exact, w.rcut_exact, w.kcut_exact)
    if w.geometry == "slab":
        A = A + slab.elastance_term(w.elec_xyz, w.box)
    return A


def build(w, A=None):
    """A and S for a workload (the once-per-geometry precompute)."""
    if A is None:
        A = elastance(w)
    return A, projected_inverse(A, sub_cell_vector(w))


class Electrostatics:
    """b, U_elyt and Coulomb forces for one workload with one k-space method.

    method 'exact'  Ewald with the converged parameters (alpha_exact, ...),
           'ewald'  Ewald with the run-time alpha, rcut, kcut,
           'pppm'   PPPM with the run-time alpha, rcut, mesh, order.
    """

    def __init__(self, w, method):
        self.w = w
        self.method = method
        if method == "pppm":
            self.G = pppm.influence(w.box, w.mesh, w.order, w.alpha)

    def b(self, site_xyz):
        b = self._b(site_xyz)
        if self.w.geometry == "slab":
            b = b + slab.b_term(self.w.elec_xyz, site_xyz, self.w.site_q, self.w.box)
        return b

    def u_elyt(self, site_xyz):
        u = self._u_elyt(site_xyz)
        if self.w.geometry == "slab":
            u = u + slab.energy_term(site_xyz, self.w.site_q, self.w.box)
        return u

    def forces(self, site_xyz, elec_q):
        f = self._forces(site_xyz, elec_q)
        if self.w.geometry == "slab":
            f = f + slab.force_term(site_xyz, self.w.site_q, self.w.elec_xyz, elec_q, self.w.box)
        return f

    def _b(self, site_xyz):
        w = self.w
        if self.method == "exact":
            return ewald.b_vector(w.elec_xyz, site_xyz, w.site_q, w.box, w.eta,
                                  w.alpha_exact, w.rcut_exact, w.kcut_exact)
        if self.method == "ewald":
            return ewald.b_vector(w.elec_xyz, site_xyz, w.site_q, w.box, w.eta,
                                  w.alpha, w.rcut, w.kcut)
        return pppm.b_vector(w.elec_xyz, site_xyz, w.site_q, w.box, w.eta, w.alpha, w.rcut,
                             w.mesh, w.order, G=self.G)

    def _u_elyt(self, site_xyz):
        w = self.w
        if self.method == "exact":
            return ewald.electrolyte_energy(site_xyz, w.site_q, w.box, w.alpha_exact,
                                            w.rcut_exact, w.kcut_exact)
        if self.method == "ewald":
            return ewald.electrolyte_energy(site_xyz, w.site_q, w.box, w.alpha, w.rcut, w.kcut)
        return pppm.electrolyte_energy(site_xyz, w.site_q, w.box, w.alpha, w.rcut,
                                       w.mesh, w.order, G=self.G)

    def _forces(self, site_xyz, elec_q):
        w = self.w
        if self.method == "exact":
            return ewald.coulomb_forces(site_xyz, w.site_q, w.elec_xyz, elec_q, w.box, w.eta,
                                        w.alpha_exact, w.rcut_exact, w.kcut_exact)
        if self.method == "ewald":
            return ewald.coulomb_forces(site_xyz, w.site_q, w.elec_xyz, elec_q, w.box, w.eta,
                                        w.alpha, w.rcut, w.kcut)
        return pppm.coulomb_forces(site_xyz, w.site_q, w.elec_xyz, elec_q, w.box, w.eta,
                                   w.alpha, w.rcut, w.mesh, w.order, G=self.G)


def field_force(w, dv):
    """Force of the applied field on the sites: F_z = -Q_j dpsi/Lz (finite field only)."""
    f = np.zeros((3, w.n_site))
    if w.geometry == "ff":
        f[2] = -w.site_q * dv / w.box[2]
    return f


def energies(w, A, q, b, u_elyt, site_xyz, dv):
    """U_coul of Eq. (3) at q and the constant-potential energy E_cp.

    U_coul = U_elyt - q.b + 1/2 q.A q.
    E_cp   = U_coul - dpsi d.q                       (doubled cell, slab)
           = U_coul - dpsi d.q + dpsi/Lz (z.q + sum_j Q_j Z_j)   (finite field)
    E_cp is stationary in q on the neutral subspace at q*, so its negative
    gradient in the site positions at fixed q is the force on the sites.
    """
    u_coul = u_elyt - q @ b + 0.5 * q @ A @ q
    d = 0.5 * w.elec_side.astype(np.float64)
    e_cp = u_coul - dv * (d @ q)
    if w.geometry == "ff":
        lz = w.box[2]
        z = w.elec_xyz[2] - lz * np.floor(w.elec_xyz[2] / lz)
        zs = site_xyz[2] - lz * np.floor(site_xyz[2] / lz)
        e_cp += dv / lz * (z @ q + w.site_q @ zs)
    return u_coul, e_cp


def step(w, A, S, es, site_xyz=None, dv=None, with_forces=True):
    """One pass of the path: R -> b -> q -> (U, E_cp, F).  Returns a dict."""
    if site_xyz is None:
        site_xyz = w.site_xyz
    if dv is None:
        dv = w.dv
    b = es.b(site_xyz)
    c = drive_vector(w)
    q = solve_charges(S, b, dv, c)
    u_elyt = es.u_elyt(site_xyz)
    u_coul, e_cp = energies(w, A, q, b, u_elyt, site_xyz, dv)
    out = dict(b=b, q=q, u_elyt=u_elyt, u_coul=u_coul, e_cp=e_cp, c=c)
    if with_forces:
        out["f"] = es.forces(site_xyz, q) + field_force(w, dv)
    return out


def loss_gradient(w, A, S, es, target, site_xyz=None, dv=None):
    """Gradient of L = sum_i (q_i - t_i)^2 + U_coul(R, q*(R)).

    dq*/dR = S db/dR and dU_coul/dq = dpsi c + (multiples of e, e1) at q*,
    so with lambda = S [2 (q - t) + dpsi c]
        dL/dR_j  = dU_elyt/dR_j - (q - lambda) . db/dR_j
                 = -(Coulomb force on site j with electrode charges q - lambda),
        dL/ddpsi = lambda . c.
    """
    if site_xyz is None:
        site_xyz = w.site_xyz
    if dv is None:
        dv = w.dv
    r = step(w, A, S, es, site_xyz, dv, with_forces=False)
    q, c = r["q"], r["c"]
    loss = np.sum((q - target) ** 2) + r["u_coul"]
    lam = S @ (2.0 * (q - target) + dv * c)
    dl_dx = -es.forces(site_xyz, q - lam)
    dl_ddv = lam @ c
    return dict(loss=loss, dl_dx=dl_dx, dl_ddv=dl_ddv, lam=lam, q=q)
