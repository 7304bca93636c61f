"""Synthetic capacitor cells: graphene electrodes and coarse-grained ions.

Everything here is input construction.  The recipe follows the paper's
model supercapacitor (Simulations section; appendix on equilibration):
graphene electrodes with 0.246 nm lattice constant whose layer nearest the
electrolyte carries the constant-potential charges, and a coarse-grained
ionic liquid with a 3-site cation (+0.4, +0.2, +0.18 e, bonds 0.3 nm) and a
1-site anion (-0.78 e).  Only the charged proximal layer of each electrode
is generated: the outer layers carry no charge and take no part in the
electrostatics.

Doubled cell (Doubled Cell Method subsection; appendix, production
paragraph): the single cell is stacked twice along z, the electrodes of the
second sub-cell are the first ones shifted by Lz with opposite polarity, and
the electrolyte of the second sub-cell is the first one mirrored about the
mid-plane of that sub-cell's electrode gap.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

WORKLOAD_NAMES = ("tiny", "paper", "large")

# Rectangular 4-atom cell of the honeycomb lattice: x along the zigzag
# direction (period a), y along the armchair direction (period 3 * bond).
_HONEYCOMB_FRAC = np.array(
    [[0.0, 0.0], [0.0, 1.0 / 3.0], [0.5, 0.5], [0.5, 5.0 / 6.0]])

MIN_SEP = 0.3          # nm, between sites of different ions and to the planes
BOND = 0.3             # nm, cation bond length
CATION_Q = (0.4, 0.2, 0.18)   # central site first, then its two neighbours
ANION_Q = -0.78


@dataclasses.dataclass
class Workload:
    """One synthetic cell plus the numerical parameters it is run with.

    Arrays use structure-of-arrays layout: ``elec_xyz`` is (3, n_elec),
    ``site_xyz`` is (3, n_site), all float64.
    """

    name: str
    geometry: str                  # "ff" (finite field), "dc" (doubled cell) or "slab"
    box: np.ndarray                # (3,) nm
    eta: float                     # Gaussian width of electrode charges, 1/nm
    # run-time splitting of the electrolyte sums
    alpha: float                   # 1/nm
    rcut: float                    # nm
    kspace: str                    # "ewald" or "pppm"
    kcut: float                    # 1/nm, explicit Ewald k-sphere (kspace == "ewald")
    mesh: tuple                    # PPPM mesh points per axis (kspace == "pppm")
    order: int                     # PPPM charge-assignment order
    # converged Ewald parameters for the elastance matrix and exact sums
    alpha_exact: float
    rcut_exact: float
    kcut_exact: float
    elec_xyz: np.ndarray
    elec_side: np.ndarray          # int8, +1 positive / -1 negative electrode
    elec_sub: Optional[np.ndarray]  # uint8, 1 = first sub-cell (dc only)
    elec_layer: Optional[np.ndarray]  # int8 graphene layer of each atom, 0 = nearest the electrolyte
    site_xyz: np.ndarray
    site_q: np.ndarray
    site_zmin: np.ndarray          # per-site z window used by the random walk
    site_zmax: np.ndarray
    mol_size: Optional[np.ndarray] = None   # sites of each molecule in site order (3: cation, 1: ion)
    lj_elec_xyz: Optional[np.ndarray] = None  # every graphene atom of the three-sheet electrodes (uncharged ones too)
    dv: float = 2.0                # V
    seed: int = 0

    @property
    def n_elec(self) -> int:
        return self.elec_xyz.shape[1]

    @property
    def n_site(self) -> int:
        return self.site_xyz.shape[1]

    def with_sites(self, site_xyz: np.ndarray) -> "Workload":
        return dataclasses.replace(self, site_xyz=np.ascontiguousarray(site_xyz, dtype=np.float64))

    def empty(self) -> "Workload":
        """The same electrodes with no electrolyte (the empty capacitor)."""
        z = np.zeros((3, 0))
        return dataclasses.replace(self, site_xyz=z, site_q=np.zeros(0),
                                   site_zmin=np.zeros(0), site_zmax=np.zeros(0))


INTERLAYER = 0.335     # nm, graphite interlayer spacing


def graphene_layer(ncell_x: int, ncell_y: int, lx: float, ly: float, z: float,
                   shifted: bool = False) -> np.ndarray:
    """Honeycomb layer of 4 * ncell_x * ncell_y atoms filling lx x ly at height z.

    shifted=True gives the B layer of A-B stacking: the lattice moved by one
    bond along the armchair direction (a third of the rectangular cell in y),
    which puts half of its atoms over hexagon centres of the A layer."""
    cx, cy = lx / ncell_x, ly / ncell_y
    dy = 1.0 / 3.0 if shifted else 0.0
    pts = []
    for iy in range(ncell_y):
        for ix in range(ncell_x):
            for fx, fy in _HONEYCOMB_FRAC:
                pts.append(((ix + fx) * cx, ((iy + fy + dy) * cy) % ly, z))
    return np.array(pts, dtype=np.float64).T.copy()


def electrode(ncell_x, ncell_y, lx, ly, z_proximal, outward, layers):
    """An electrode of `layers` graphene sheets in A-B-A stacking: the first at
    z_proximal (facing the electrolyte), the others INTERLAYER apart going
    `outward` (-1: down, +1: up).  Returns (xyz, layer index per atom)."""
    xyz, lay = [], []
    for k in range(layers):
        xyz.append(graphene_layer(ncell_x, ncell_y, lx, ly, z_proximal + outward * k * INTERLAYER,
                                  shifted=(k % 2 == 1)))
        lay.append(np.full(xyz[-1].shape[1], k, np.int8))
    return np.concatenate(xyz, axis=1), np.concatenate(lay)


def _random_unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _min_dist2(p: np.ndarray, placed: np.ndarray, lx: float, ly: float) -> float:
    """Smallest squared distance from p (3,) to placed (n, 3), periodic in x and y."""
    if placed.shape[0] == 0:
        return np.inf
    d = placed - p
    d[:, 0] -= lx * np.round(d[:, 0] / lx)
    d[:, 1] -= ly * np.round(d[:, 1] / ly)
    return float(np.min(np.einsum("ij,ij->i", d, d)))


def random_electrolyte(rng, n_pairs, lx, ly, zmin, zmax, cation_sites):
    """Random sequential placement of n_pairs cations and anions.

    cation_sites == 1 gives single-site cations of +0.78 e; 3 gives the rigid
    3-site chain (central site +0.4, neighbours +0.2 and +0.18, bonds 0.3 nm,
    120 degree angle).  Sites of different ions stay >= 0.3 nm apart and all
    sites lie in [zmin, zmax].
    """
    cap = n_pairs * (cation_sites + 1)
    placed = np.zeros((cap, 3))
    charges = np.zeros(cap)
    n = 0
    for k in range(2 * n_pairs):
        is_cation = (k % 2 == 0)
        for attempt in range(200000):
            c = np.array([rng.uniform(0, lx), rng.uniform(0, ly), rng.uniform(zmin, zmax)])
            if is_cation and cation_sites == 3:
                u = _random_unit(rng)
                w = _random_unit(rng)
                w -= u * np.dot(u, w)
                w /= np.linalg.norm(w)
                b = c + BOND * u
                cc = c + BOND * (math.cos(2 * math.pi / 3) * u + math.sin(2 * math.pi / 3) * w)
                sites = np.stack([c, b, cc])
                qs = CATION_Q
            else:
                sites = c[None, :]
                qs = (0.78,) if is_cation else (ANION_Q,)
            if np.any(sites[:, 2] < zmin) or np.any(sites[:, 2] > zmax):
                continue
            if all(_min_dist2(s, placed[:n], lx, ly) >= MIN_SEP ** 2 for s in sites):
                break
        else:
            raise RuntimeError("random placement did not converge")
        for s, q in zip(sites, qs):
            s = s.copy()
            s[0] %= lx
            s[1] %= ly
            placed[n] = s
            charges[n] = q
            n += 1
    return placed[:n].T.copy(), charges[:n].copy()


def molecule_sizes(site_q: np.ndarray) -> np.ndarray:
    """Sites per molecule in site order: a 3-site cation starts with its +0.4 e
    central site; every other site is an ion of its own."""
    sizes, j = [], 0
    while j < site_q.size:
        k = 3 if abs(site_q[j] - CATION_Q[0]) < 1e-12 else 1
        sizes.append(k)
        j += k
    return np.array(sizes, dtype=np.int32)


def _double(w: Workload, z_lo: float, z_hi: float) -> Workload:
    """Doubled-cell construction from a single finite-field style cell."""
    lz = w.box[2]
    e2 = w.elec_xyz.copy()
    e2[2] += lz
    s2 = w.site_xyz.copy()
    s2[2] = lz + (z_lo + z_hi) - s2[2]
    box = w.box.copy()
    box[2] = 2 * lz
    mesh = (w.mesh[0], w.mesh[1], 2 * w.mesh[2])
    zmin2 = lz + (z_lo + z_hi) - w.site_zmax
    zmax2 = lz + (z_lo + z_hi) - w.site_zmin
    return dataclasses.replace(
        w, geometry="dc", box=box, mesh=mesh,
        elec_xyz=np.concatenate([w.elec_xyz, e2], axis=1),
        elec_side=np.concatenate([w.elec_side, -w.elec_side]).astype(np.int8),
        elec_sub=np.concatenate([np.ones(w.n_elec, np.uint8), np.zeros(w.n_elec, np.uint8)]),
        elec_layer=np.concatenate([w.elec_layer, w.elec_layer]),
        site_xyz=np.concatenate([w.site_xyz, s2], axis=1),
        site_q=np.concatenate([w.site_q, w.site_q]),
        site_zmin=np.concatenate([w.site_zmin, zmin2]),
        site_zmax=np.concatenate([w.site_zmax, zmax2]),
        mol_size=np.concatenate([w.mol_size, w.mol_size]),
        lj_elec_xyz=np.concatenate([w.lj_elec_xyz, w.lj_elec_xyz + np.array([[0.0], [0.0], [lz]])], axis=1),
    )


SLAB_FACTOR = 3.0   # periodic length over the cell's length in slab geometry


def _slab(w: Workload, factor: float) -> Workload:
    """Slab geometry: the same cell in the middle of a z-period `factor` times
    as long (empty space of equal depth below and above it, across z = 0),
    and the mesh lengthened in z in proportion (same spacing)."""
    box = w.box.copy()
    box[2] = factor * w.box[2]
    kz = int(round(factor * w.mesh[2]))
    dz = 0.5 * (box[2] - w.box[2])
    ex, sx, lj = w.elec_xyz.copy(), w.site_xyz.copy(), w.lj_elec_xyz.copy()
    ex[2] += dz
    sx[2] += dz
    lj[2] += dz
    return dataclasses.replace(w, geometry="slab", box=box, mesh=(w.mesh[0], w.mesh[1], kz),
                               elec_xyz=ex, site_xyz=sx, site_zmin=w.site_zmin + dz, site_zmax=w.site_zmax + dz,
                               lj_elec_xyz=lj)


def make_workload(name: str, geometry: str = "ff", seed: Optional[int] = None, layers: int = 1,
                  slab_factor: float = SLAB_FACTOR) -> Workload:
    """Build one of the named workloads ('tiny', 'paper', 'large') in 'ff', 'dc' or 'slab'.

    Slab geometry (the non-periodic setting the paper compares against) keeps
    the finite-field cell's contents and puts them in a z-period slab_factor
    times as long (vacuum above the upper electrode), as the slab correction
    needs.

    layers = 1 charges only the graphene sheet of each electrode nearest the
    electrolyte (the production setting of the paper); layers = 3 charges all
    three sheets (A-B-A stacking, 0.335 nm apart), as in the paper's re-runs
    of snapshots.  The electrolyte is the same in both."""
    if geometry not in ("ff", "dc", "slab"):
        raise ValueError("geometry must be 'ff', 'dc' or 'slab'")
    if layers not in (1, 3):
        raise ValueError("layers must be 1 or 3")
    eta = 19.79
    if name == "tiny":
        a = 0.246
        lx, ly, lz = 6 * a, 1.27824, 6.0
        # with three sheets the whole system moves up by two spacings, so the
        # cell boundary z = 0 stays behind the lower electrode (a finite-field
        # electrode must not cross it)
        z_lo = 2 * INTERLAYER if layers == 3 else 0.0
        z_hi = z_lo + 4.34
        lo, lo_l = electrode(6, 3, lx, ly, z_lo, -1, 3)
        hi, hi_l = electrode(6, 3, lx, ly, z_hi, +1, 3)
        seed = 1 if seed is None else seed
        rng = np.random.default_rng(seed)
        sxyz, sq = random_electrolyte(rng, 50, lx, ly, z_lo + MIN_SEP, z_hi - MIN_SEP, 1)
        params = dict(alpha=2.97, rcut=1.2, kspace="ewald", kcut=24.0, mesh=(16, 16, 64), order=5,
                      alpha_exact=2.97, rcut_exact=2.0, kcut_exact=33.0)
    elif name in ("paper", "large"):
        reps = 1 if name == "paper" else 2
        lx = ly = 3.4 * reps
        lz = 12.625
        z_lo, z_hi = 1.3125, 11.3125
        lo, lo_l = electrode(11 * reps, 10 * reps, lx, ly, z_lo, -1, 3)
        hi, hi_l = electrode(11 * reps, 10 * reps, lx, ly, z_hi, +1, 3)
        seed = (2 if name == "paper" else 3) if seed is None else seed
        rng = np.random.default_rng(seed)
        sxyz, sq = random_electrolyte(rng, 320 * reps * reps, lx, ly,
                                      z_lo + MIN_SEP, z_hi - MIN_SEP, 3)
        if name == "paper":
            params = dict(alpha=2.21, rcut=1.2, kspace="pppm", kcut=0.0, mesh=(18, 18, 64), order=5,
                          alpha_exact=2.21, rcut_exact=2.7, kcut_exact=24.5)
        else:
            params = dict(alpha=2.21, rcut=1.2, kspace="pppm", kcut=0.0, mesh=(36, 36, 64), order=5,
                          alpha_exact=1.6, rcut_exact=3.7, kcut_exact=17.5)
    else:
        raise ValueError(f"unknown workload {name!r}")
    # all three sheets take part in the Lennard-Jones interactions; the
    # constant-potential charges sit on the nearest sheet only (layers = 1) or
    # on all three
    lj_all = np.concatenate([lo, hi], axis=1)
    keep_lo, keep_hi = lo_l < layers, hi_l < layers
    lo, lo_l, hi, hi_l = lo[:, keep_lo], lo_l[keep_lo], hi[:, keep_hi], hi_l[keep_hi]
    n_half = lo.shape[1]
    w = Workload(
        name=name, geometry="ff", box=np.array([lx, ly, lz]), eta=eta,
        elec_xyz=np.concatenate([lo, hi], axis=1),
        elec_side=np.concatenate([-np.ones(n_half, np.int8), np.ones(n_half, np.int8)]),
        elec_sub=None, elec_layer=np.concatenate([lo_l, hi_l]), site_xyz=sxyz, site_q=sq,
        site_zmin=np.full(sq.shape, z_lo + MIN_SEP), site_zmax=np.full(sq.shape, z_hi - MIN_SEP),
        mol_size=molecule_sizes(sq), lj_elec_xyz=lj_all,
        seed=seed, **params)
    if geometry == "dc":
        w = _double(w, z_lo, z_hi)
    elif geometry == "slab":
        w = _slab(w, slab_factor)
    return w


def random_walk(w: Workload, n_steps: int, sigma: float = 0.005, seed: int = 12345) -> np.ndarray:
    """Trajectory of n_steps frames, (n_steps, 3, n_site).

    Each step adds N(0, sigma^2) to every coordinate; x and y wrap, and a
    site whose new z would leave its window [site_zmin, site_zmax] keeps
    its old position for that step.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n_steps, 3, w.n_site))
    cur = w.site_xyz.copy()
    for t in range(n_steps):
        new = cur + rng.normal(0.0, sigma, size=cur.shape)
        bad = (new[2] < w.site_zmin) | (new[2] > w.site_zmax)
        new[:, bad] = cur[:, bad]
        new[0] %= w.box[0]
        new[1] %= w.box[1]
        out[t] = new
        cur = new
    return out


def perturbed_frames(w: Workload, n_frames: int, sigma: float = 0.05, seed: int = 4) -> np.ndarray:
    """n_frames independent Gaussian perturbations of the base sites, wrapped into the cell."""
    rng = np.random.default_rng(seed)
    out = w.site_xyz[None, :, :] + rng.normal(0.0, sigma, size=(n_frames, 3, w.n_site))
    out %= w.box[None, :, None]
    return out


# --------------------------------------------------------------------------
# molecular dynamics inputs
# --------------------------------------------------------------------------

# Synthetic stand-ins for the coarse-grained ionic liquid and graphene force
# fields (the paper takes them from the literature, which is not at hand):
# masses of the three cation sites and the anion (a 139 + 145 amu ion pair),
# Lennard-Jones sigma (nm) and epsilon (kJ/mol) per site kind, graphene
# carbon, Lorentz-Berthelot combination.  sigma is kept near the 0.3 nm
# placement separation so that the seeded configurations start without
# overlaps.
CATION_MASS = (67.0, 15.0, 57.0)
ANION_MASS = 145.0
SINGLE_CATION_MASS = 139.0
SITE_SIGMA, SITE_EPS = 0.30, 1.5
CARBON_SIGMA, CARBON_EPS, CARBON_MASS = 0.34, 0.23, 12.011
LJ_CUT = 1.6              # nm (appendix: non-Coulombic cutoff 16 A)
MD_DT = 0.002             # ps (2 fs)
MD_TEMPERATURE = 400.0    # K
MD_TAU = 0.1              # ps, Nose-Hoover time constant
MD_CHARGE_EVERY = 5       # charge update every 5 steps


@dataclasses.dataclass
class MDSetup:
    """Inputs of the constant-potential MD loop for one workload."""

    site_mass: np.ndarray          # (n_site,) amu
    site_sigma: np.ndarray         # (n_site,) nm
    site_eps: np.ndarray           # (n_site,) kJ/mol
    lj_elec_xyz: np.ndarray        # (3, n) every graphene atom (all sheets), fixed
    carbon_sigma: float
    carbon_eps: float
    lj_cut: float
    mol_size: np.ndarray           # (n_mol,) 3 (rigid cation) or 1
    mol_group: np.ndarray          # (n_mol,) thermostat group (doubled cell: one per sub-cell)
    n_groups: int
    bond: float                    # cation bond length (nm); the third side is bond * sqrt(3)
    dt: float
    temperature: float
    tau: float
    charge_every: int


def md_setup(w: Workload) -> MDSetup:
    """Force field, rigid molecules and thermostat groups for a workload; the
    Lennard-Jones electrodes are all three sheets of each electrode whatever
    the workload charges."""
    sizes = w.mol_size
    mass = np.empty(w.n_site)
    j = 0
    for k in sizes:
        if k == 3:
            mass[j:j + 3] = CATION_MASS
        else:
            mass[j] = ANION_MASS if w.site_q[j] < 0 else SINGLE_CATION_MASS
        j += k
    n_mol = sizes.size
    if w.geometry == "dc":
        groups = np.concatenate([np.zeros(n_mol // 2, np.int32), np.ones(n_mol - n_mol // 2, np.int32)])
        n_groups = 2
    else:
        groups = np.zeros(n_mol, np.int32)
        n_groups = 1
    lj = w.lj_elec_xyz
    return MDSetup(site_mass=mass, site_sigma=np.full(w.n_site, SITE_SIGMA), site_eps=np.full(w.n_site, SITE_EPS),
                   lj_elec_xyz=np.ascontiguousarray(lj), carbon_sigma=CARBON_SIGMA, carbon_eps=CARBON_EPS,
                   lj_cut=LJ_CUT, mol_size=sizes, mol_group=groups, n_groups=n_groups, bond=BOND, dt=MD_DT,
                   temperature=MD_TEMPERATURE, tau=MD_TAU, charge_every=MD_CHARGE_EVERY)
