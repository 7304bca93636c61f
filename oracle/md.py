"""The constant-potential MD loop (appendix, force-field and production
paragraphs): velocity Verlet with a 2 fs step, a Nose-Hoover thermostat on
the electrolyte (one per sub-cell in the doubled cell), rigid three-site
cations held by SHAKE (with its velocity counterpart RATTLE), Lennard-Jones
site-site and site-graphene interactions within 1.6 nm, and the electrode
charges re-solved every fifth step (between updates the forces use the last
charges).

Units: nm, ps, amu, kJ/mol (forces kJ/mol/nm); the electrostatics of
``cpm`` are in eV and converted with EV_KJ.

One step, from positions x, velocities v and forces F (the
Nose-Hoover half steps follow the usual symmetric splitting of a single
thermostat variable xi per group with conjugate position eta):

    thermostat half step; v += (dt/2) F/m
    x_new = x + dt v, then SHAKE to the constraint lengths; v = (x_new - x)/dt
    F = forces(x_new)              (charges re-solved on every k-th step)
    v += (dt/2) F/m; RATTLE (velocities normal to the constraints)
    thermostat half step

thermostat half step (per group, Q = N_f k T tau^2, K2 = sum m v^2):
    xi += (dt/4)(K2 - N_f k T)/Q; eta += (dt/2) xi; v *= exp(-xi dt/2);
    K2 *= exp(-xi dt); xi += (dt/4)(K2 - N_f k T)/Q

The extended energy KE + U + sum_g (Q_g xi_g^2 / 2 + N_f,g k T eta_g) is
conserved by the exact dynamics (with charges solved every step).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import cpm

EV_KJ = 96.48533212          # kJ/mol per eV
KB = 0.0083144626            # kJ/mol/K


def min_image(d, box):
    return d - box[:, None] * np.round(d / box[:, None])


@dataclasses.dataclass
class Constraints:
    """Rigid molecules as distance constraints (i, j, length)."""
    i: np.ndarray
    j: np.ndarray
    d: np.ndarray


def rigid_constraints(mol_size, bond):
    """Three distances per three-site molecule: two bonds and the third side
    of the 120-degree triangle (bond * sqrt(3))."""
    ii, jj, dd = [], [], []
    start = 0
    for k in mol_size:
        if k == 3:
            ii += [start, start, start + 1]
            jj += [start + 1, start + 2, start + 2]
            dd += [bond, bond, bond * math.sqrt(3.0)]
        start += k
    return Constraints(np.array(ii, int), np.array(jj, int), np.array(dd))


def shake(x, x_old, m, con, box, tol=1e-13, max_iter=500):
    """Move x along the old constraint vectors until every |x_i - x_j| = d."""
    x = x.copy()
    for _ in range(max_iter):
        done = True
        for i, j, d in zip(con.i, con.j, con.d):
            r = min_image((x[:, i] - x[:, j])[:, None], box)[:, 0]
            diff = d * d - r @ r
            if abs(diff) > tol * d * d:
                done = False
                ro = min_image((x_old[:, i] - x_old[:, j])[:, None], box)[:, 0]
                g = diff / (2.0 * (ro @ r) * (1.0 / m[i] + 1.0 / m[j]))
                x[:, i] += g * ro / m[i]
                x[:, j] -= g * ro / m[j]
        if done:
            return x
    raise RuntimeError("SHAKE did not converge")


def rattle(v, x, m, con, box, tol=1e-13, max_iter=500):
    """Remove the velocity components along every constraint."""
    v = v.copy()
    for _ in range(max_iter):
        done = True
        for i, j, d in zip(con.i, con.j, con.d):
            r = min_image((x[:, i] - x[:, j])[:, None], box)[:, 0]
            vr = (v[:, i] - v[:, j]) @ r
            if abs(vr) > tol * d * (np.abs(v[:, i]).max() + np.abs(v[:, j]).max() + 1e-300):
                done = False
                k = vr / (d * d * (1.0 / m[i] + 1.0 / m[j]))
                v[:, i] -= k * r / m[i]
                v[:, j] += k * r / m[j]
        if done:
            return v
    raise RuntimeError("RATTLE did not converge")


def lj_forces(x, setup, box):
    """Lennard-Jones forces and energy: site-site pairs of different molecules
    and every site with every graphene atom, cut at lj_cut (energy shifted to
    zero there), Lorentz-Berthelot combination."""
    n = x.shape[1]
    mol = np.repeat(np.arange(setup.mol_size.size), setup.mol_size)
    f = np.zeros((3, n))
    u = 0.0
    rc2 = setup.lj_cut ** 2

    def pair_terms(d, sig, eps):
        r2 = np.einsum("kab,kab->ab", d, d)
        inside = (r2 < rc2) & (r2 > 0.0)
        r2s = np.where(inside, r2, 1.0)
        s6 = (sig * sig / r2s) ** 3
        sc6 = (sig * sig / rc2) ** 3
        e = np.where(inside, 4 * eps * (s6 * s6 - s6) - 4 * eps * (sc6 * sc6 - sc6), 0.0)
        fr = np.where(inside, 24 * eps * (2 * s6 * s6 - s6) / r2s, 0.0)     # F = fr * d
        return e, fr

    d = min_image((x[:, :, None] - x[:, None, :]).reshape(3, -1), box).reshape(3, n, n)
    sig = 0.5 * (setup.site_sigma[:, None] + setup.site_sigma[None, :])
    eps = np.sqrt(setup.site_eps[:, None] * setup.site_eps[None, :])
    e, fr = pair_terms(d, sig, eps)
    other = mol[:, None] != mol[None, :]
    e = np.where(other, e, 0.0)
    fr = np.where(other, fr, 0.0)
    u += 0.5 * e.sum()
    f += np.einsum("kab,ab->ka", d, fr)
    c = setup.lj_elec_xyz
    d = min_image((x[:, :, None] - c[:, None, :]).reshape(3, -1), box).reshape(3, n, c.shape[1])
    sig = 0.5 * (setup.site_sigma[:, None] + setup.carbon_sigma)
    eps = np.sqrt(setup.site_eps[:, None] * setup.carbon_eps)
    e, fr = pair_terms(d, sig, eps)
    u += e.sum()
    f += np.einsum("kab,ab->ka", d, fr)
    return f, u


def verlet_step(x, v, f, m, con, box, dt, force, thermo=None):
    """One velocity-Verlet step with constraints, (x, v, f) -> (x', v', f'):
    force(x) gives the forces at x; thermo(v) (if given) is the thermostat's
    half step, applied before the first kick and after the second."""
    if thermo is not None:
        v = thermo(v)
    v = v + 0.5 * dt * f / m
    x_new = shake(x + dt * v, x, m, con, box)
    v = (x_new - x) / dt
    f = force(x_new)
    v = v + 0.5 * dt * f / m
    v = rattle(v, x_new, m, con, box)
    if thermo is not None:
        v = thermo(v)
    return x_new, v, f


@dataclasses.dataclass
class State:
    x: np.ndarray
    v: np.ndarray
    f: np.ndarray
    q: np.ndarray
    xi: np.ndarray
    eta: np.ndarray
    step: int
    u_lj: float
    e_cp: float


class Loop:
    """The MD loop for one workload: w, A, S and the electrostatics method of
    the oracle, the MD inputs (workloads.md_setup) and dV."""

    def __init__(self, w, A, S, method, setup, dv, thermostat=True):
        self.w, self.A, self.S, self.setup, self.dv = w, A, S, setup, dv
        self.thermostat = thermostat
        self.es = cpm.Electrostatics(w, method)
        self.m = setup.site_mass
        self.con = rigid_constraints(setup.mol_size, setup.bond)
        mol = np.repeat(np.arange(setup.mol_size.size), setup.mol_size)
        self.site_group = setup.mol_group[mol]
        self.kt = KB * setup.temperature
        self.nf = np.zeros(setup.n_groups)
        for g in range(setup.n_groups):
            sel = self.site_group == g
            ncon = np.sum(self.site_group[self.con.i] == g)
            self.nf[g] = 3 * sel.sum() - ncon
        self.Q = self.nf * self.kt * setup.tau ** 2

    def forces(self, x, q):
        """Total force (kJ/mol/nm), new or given electrode charges, U_LJ, E_cp."""
        f_lj, u_lj = lj_forces(x, self.setup, self.w.box)
        if q is None:
            r = cpm.step(self.w, self.A, self.S, self.es, site_xyz=x, dv=self.dv)
            return f_lj + EV_KJ * r["f"], r["q"], u_lj, r["e_cp"]
        fc = self.es.forces(x, q) + cpm.field_force(self.w, self.dv)
        return f_lj + EV_KJ * fc, q, u_lj, None

    def start(self, x, v):
        """Initial state: velocities made normal to the constraints, forces with fresh charges."""
        v = rattle(v, x, self.m, self.con, self.w.box)
        f, q, u, e = self.forces(x, None)
        ng = self.setup.n_groups
        return State(x.copy(), v, f, q, np.zeros(ng), np.zeros(ng), 0, u, e)

    def thermostat_half(self, s, v):
        """The thermostat's half step on velocities v (returned scaled); xi and eta of s advance."""
        dt = self.setup.dt
        v = v.copy()
        for g in range(self.setup.n_groups):
            sel = self.site_group == g
            k2 = np.sum(self.m[sel] * np.sum(v[:, sel] ** 2, axis=0))
            s.xi[g] += 0.25 * dt * (k2 - self.nf[g] * self.kt) / self.Q[g]
            s.eta[g] += 0.5 * dt * s.xi[g]
            scale = math.exp(-0.5 * dt * s.xi[g])
            v[:, sel] *= scale
            k2 *= scale * scale
            s.xi[g] += 0.25 * dt * (k2 - self.nf[g] * self.kt) / self.Q[g]
        return v

    def step(self, s):
        s.step += 1
        update = s.step % self.setup.charge_every == 0
        box = self.w.box

        def force(x):
            f, q, u, e = self.forces(x, None if update else s.q)
            s.q, s.u_lj = q, u
            if update:
                s.e_cp = e
            return f

        thermo = (lambda v: self.thermostat_half(s, v)) if self.thermostat else None
        s.x, s.v, s.f = verlet_step(s.x, s.v, s.f, self.m, self.con, box, self.setup.dt, force, thermo)
        return s

    def kinetic(self, s):
        return 0.5 * np.sum(self.m * np.sum(s.v ** 2, axis=0))

    def extended_energy(self, s, e_cp):
        """KE + U_LJ + E_cp (kJ/mol) + the thermostat terms."""
        th = np.sum(0.5 * self.Q * s.xi ** 2 + self.nf * self.kt * s.eta)
        return self.kinetic(s) + s.u_lj + EV_KJ * e_cp + th
