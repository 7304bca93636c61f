"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, brute-force sums written here from scratch, invariances the method
must have, finite differences and a textbook lattice constant.
"""

import dataclasses
import functools
import math

import numpy as np
import pytest

from conftest import built, workload
from oracle import KE, cells, cpm, ewald, pppm, slab

EPS0 = 1.0 / (4.0 * math.pi * KE)


# --------------------------------------------------------------------------
# helpers written independently of the oracle
# --------------------------------------------------------------------------

def honeycomb_seff(cx, cy, eta, nmax=60):
    """Effective Gaussian offset of a charged honeycomb layer.

    The potential of a periodic layer of identical Gaussian charges at one of
    its own atoms, relative to an ideal sheet of the same areal charge, is
    -(sigma / 2 eps0) s_eff with
      s_eff = sqrt(2/pi)/eta - (1/n_b) sum_{G != 0} S_A(G) erfc(|G|/(sqrt2 eta))/|G|,
    G over the 2D reciprocal lattice of the rectangular cell cx x cy with
    n_b = 4 basis atoms and S_A(G) = sum_b cos(G.(r_A - r_b)).
    """
    basis = np.array([[0, 0], [0, 1 / 3], [0.5, 0.5], [0.5, 5 / 6]]) * [cx, cy]
    i, j = np.meshgrid(np.arange(-nmax, nmax + 1), np.arange(-nmax, nmax + 1), indexing="ij")
    G = np.stack([2 * math.pi * i / cx, 2 * math.pi * j / cy], -1).reshape(-1, 2)
    g = np.linalg.norm(G, axis=1)
    keep = g > 0
    G, g = G[keep], g[keep]
    SA = np.cos((basis[0] - basis) @ G.T).sum(axis=0)
    from scipy.special import erfc
    return math.sqrt(2 / math.pi) / eta - np.sum(SA * erfc(g / (math.sqrt(2) * eta)) / g) / 4


def empty_charges(w, A, S, dv):
    return S @ (dv * cpm.drive_vector(w))


# --------------------------------------------------------------------------
# P5 / P6: the empty capacitor
# --------------------------------------------------------------------------

def test_empty_capacitor_closed_form():
    """Empty parallel-plate capacitor of Gaussian graphene layers (Eq. 8, 11, 14).

    Doubled cell: Q+ = eps0 A dpsi/(g - s_eff); finite field:
    Q+ = eps0 A dpsi/(g - s_eff Lz/(Lz - g)).  Every atom of a layer carries
    the same charge by symmetry.
    """
    dv = 2.0
    w, A, S = built("tiny", "ff")
    seff = honeycomb_seff(w.box[0] / 6, w.box[1] / 3, w.eta)
    assert abs(seff - 0.03216) < 5e-6
    area = w.box[0] * w.box[1]
    g, lz = 4.34, w.box[2]
    q = empty_charges(w, A, S, dv)
    up = w.elec_side > 0
    qff = EPS0 * area * dv / (g - seff * lz / (lz - g))
    assert abs(q[up].sum() - qff) < 1e-10 * qff
    assert np.ptp(q[up]) < 1e-12 * abs(q[up].mean())
    assert np.ptp(q[~up]) < 1e-12 * abs(q[~up].mean())

    wd, Ad, Sd = built("tiny", "dc")
    qd = empty_charges(wd, Ad, Sd, dv)
    qdc = EPS0 * area * dv / (g - seff)
    for sub in (0, 1):
        for side in (-1, 1):
            m = (wd.elec_sub == sub) & (wd.elec_side == side)
            assert abs(qd[m].sum() - side * qdc) < 1e-10 * qdc
            assert np.ptp(qd[m]) < 1e-12 * qdc
    # finite-field / doubled-cell ratio (not 1 for Gaussian electrodes)
    ratio = (g - seff) / (g - seff * lz / (lz - g))
    assert abs(q[up].sum() / qd[(wd.elec_sub == 1) & (wd.elec_side > 0)].sum() - ratio) < 1e-9


def test_ff_dc_mismatch_shrinks_with_lz():
    """The FF/DC ratio (g - s)/(g - s Lz/(Lz - g)) tends to 1 as the back region grows."""
    w0 = workload("tiny", "ff")
    seff = honeycomb_seff(w0.box[0] / 6, w0.box[1] / 3, w0.eta)
    g = 4.34
    prev = None
    for lz in (6.0, 9.0):
        w = dataclasses.replace(w0, box=np.array([w0.box[0], w0.box[1], lz])).empty()
        A, S = cpm.build(w)
        q = empty_charges(w, A, S, 2.0)[w.elec_side > 0].sum()
        qdc = EPS0 * w.box[0] * w.box[1] * 2.0 / (g - seff)
        mismatch = q / qdc - 1.0
        assert abs(mismatch - ((g - seff) / (g - seff * lz / (lz - g)) - 1)) < 1e-9
        if prev is not None:
            assert mismatch < prev
        prev = mismatch


def test_ff_dc_agreement_with_electrolyte():
    """Filled cell: finite field against the first sub-cell of the doubled cell.

    * The net charge of each electrode is set by the laterally averaged
      (one-dimensional) part of the electrostatics, where the empty-capacitor
      ratio (g - s)/(g - s Lz/(Lz - g)) applies to the electrolyte-induced
      charge as well; the two geometries' net charges stand in that ratio at
      dpsi = 0 and 2 V.
    * The in-plane charge pattern (charges minus their electrode's mean) is
      the same in both up to the small influence of the second sub-cell
      through the electrodes (screening, Doubled Cell Method subsection).
    * The doubled cell is mirror-symmetric about the plane between the
      sub-cells (electrolyte mirrored, polarity reversed), so each atom of the
      second sub-cell carries the charge of its mirror atom in the first.
    """
    wf, Af, Sf = built("tiny", "ff")
    wd, Ad, Sd = built("tiny", "dc")
    n = wf.n_elec
    seff = honeycomb_seff(wf.box[0] / 6, wf.box[1] / 3, wf.eta)
    g, lz = 4.34, wf.box[2]
    ratio = (g - seff) / (g - seff * lz / (lz - g))
    up = wf.elec_side > 0
    half = n // 2
    for dv in (0.0, 2.0):
        qf = cpm.step(wf, Af, Sf, cpm.Electrostatics(wf, "exact"), dv=dv, with_forces=False)["q"]
        qd = cpm.step(wd, Ad, Sd, cpm.Electrostatics(wd, "exact"), dv=dv, with_forces=False)["q"]
        q1, q2 = qd[:n], qd[n:]
        assert abs(qf[up].sum() / q1[up].sum() - ratio) < 5e-5
        assert abs(qf[~up].sum() / q1[~up].sum() - ratio) < 5e-5
        for m in (up, ~up):
            a, b = qf[m] - qf[m].mean(), q1[m] - q1[m].mean()
            assert np.abs(a - b).max() < 1e-3 * np.abs(a).max()
        # mirror: sub-cell 1 upper layer <-> sub-cell 2 lower layer (same x, y)
        assert np.abs(q2[:half] - q1[half:]).max() < 1e-12
        assert np.abs(q2[half:] - q1[:half]).max() < 1e-12


# --------------------------------------------------------------------------
# P1 / P2 / P7: constraint algebra
# --------------------------------------------------------------------------

@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_kkt_residual_and_neutrality(geometry):
    """A q* - v lies in span(e) (and e1 for the doubled cell); e.q* = 0 (Eq. 5-7, 12)."""
    w, A, S = built("tiny", geometry)
    es = cpm.Electrostatics(w, "ewald")
    r = cpm.step(w, A, S, es, with_forces=False)
    q, b, c = r["q"], r["b"], r["c"]
    v = b + w.dv * c
    res = A @ q - v
    basis = [np.ones(w.n_elec)]
    if geometry == "dc":
        basis.append(w.elec_sub.astype(float))
    B = np.stack(basis, 1)
    coef, *_ = np.linalg.lstsq(B, res, rcond=None)
    assert np.abs(res - B @ coef).max() < 1e-10 * np.abs(v - v.mean()).max()
    assert abs(q.sum()) < 1e-12
    if geometry == "dc":
        assert abs(q[w.elec_sub == 1].sum()) < 1e-12
    # S is symmetric, annihilates e (and e1), and is a generalised inverse of A
    assert np.abs(S - S.T).max() < 1e-14 * np.abs(S).max()
    assert np.abs(S @ np.ones(w.n_elec)).max() < 1e-13 * np.abs(S).max()
    assert np.abs(S @ A @ S - S).max() < 1e-10 * np.abs(S).max()
    P = A @ S
    assert np.abs(P @ P - P).max() < 1e-10
    # U_coul identity: 1/2 q.A q = 1/2 q.v at q*
    assert abs(q @ A @ q - q @ v) < 1e-12 * abs(q @ v)


def test_linear_in_dv():
    """q*(dpsi) = q*(0) + dpsi S c exactly (Eq. 8 and 11 are affine in dpsi)."""
    w, A, S = built("tiny", "ff")
    es = cpm.Electrostatics(w, "ewald")
    q0 = cpm.step(w, A, S, es, dv=0.0, with_forces=False)["q"]
    for dv in (0.7, 2.0, -1.3):
        q = cpm.step(w, A, S, es, dv=dv, with_forces=False)["q"]
        assert np.abs(q - (q0 + dv * S @ cpm.drive_vector(w))).max() < 1e-14


# --------------------------------------------------------------------------
# P3: invariances
# --------------------------------------------------------------------------

def test_invariances():
    w, A, S = built("tiny", "ff")
    es = cpm.Electrostatics(w, "ewald")
    r = cpm.step(w, A, S, es)
    q = r["q"]
    e = np.ones(w.n_elec)
    c = cpm.drive_vector(w)
    # b + const e, A + const e e^T, z -> z + const (drive vector shifts by a multiple of e)
    assert np.abs(S @ (r["b"] + 3.7 * e + w.dv * c) - q).max() < 1e-13
    S2 = cpm.projected_inverse(A + 5.0 * np.outer(e, e))
    assert np.abs(S2 - S).max() < 1e-12 * np.abs(S).max()
    assert np.abs(S @ (r["b"] + w.dv * (c - 0.25 * e)) - q).max() < 1e-13
    # lattice translation in x and y of the whole system
    shift = np.array([0.31, -0.17, 0.0])[:, None]
    wt = dataclasses.replace(w, elec_xyz=(w.elec_xyz + shift) % w.box[:, None])
    At, St = cpm.build(wt)
    rt = cpm.step(wt, At, St, cpm.Electrostatics(wt, "ewald"), site_xyz=(w.site_xyz + shift) % w.box[:, None])
    assert np.abs(rt["q"] - q).max() < 1e-10
    assert np.abs(rt["f"] - r["f"]).max() < 1e-9 * np.abs(r["f"]).max()
    assert abs(rt["u_coul"] - r["u_coul"]) < 1e-10 * abs(r["u_coul"])


def test_alpha_independence():
    """Converged Ewald results do not depend on the splitting parameter."""
    w, A, S = built("tiny", "ff")
    res = []
    for alpha, rcut, kcut in ((2.97, 2.0, 33.0), (4.0, 1.5, 44.0)):
        wa = dataclasses.replace(w, alpha_exact=alpha, rcut_exact=rcut, kcut_exact=kcut)
        Aa, Sa = cpm.build(wa)
        res.append((Aa, cpm.step(wa, Aa, Sa, cpm.Electrostatics(wa, "exact"))))
    (A1, r1), (A2, r2) = res
    # A changes by the rank-one constant k_e (pi/V)(1/alpha^2 - 2/eta^2) e e^T
    vol = np.prod(w.box)
    const = KE * math.pi / vol * ((1 / 2.97 ** 2 - 1 / 4.0 ** 2))
    assert np.abs((A1 - A2) - const).max() < 1e-10 * np.abs(A1).max()
    assert np.abs(r1["q"] - r2["q"]).max() < 1e-11
    assert np.abs(r1["f"] - r2["f"]).max() < 1e-9 * np.abs(r1["f"]).max()
    assert abs(r1["u_coul"] - r2["u_coul"]) < 1e-10 * abs(r1["u_coul"])


# --------------------------------------------------------------------------
# P4: brute-force reciprocal sums without splitting
# --------------------------------------------------------------------------

def _all_k(box, kcut):
    nmax = [int(kcut * L / (2 * math.pi)) for L in box]
    n = np.stack(np.meshgrid(*[np.arange(-m, m + 1) for m in nmax], indexing="ij"), -1).reshape(-1, 3)
    k = 2 * math.pi * n / np.asarray(box)
    k2 = (k * k).sum(1)
    keep = (k2 > 0) & (k2 <= kcut ** 2)
    return k[keep], k2[keep]


def test_bruteforce_reciprocal_tiny_cell():
    """A and b as plain Fourier sums of the Gaussian interactions (no real space).

    Gaussian-Gaussian: (4 pi/V) sum_k exp(-k^2/2eta^2)/k^2 cos(k.r);
    point-Gaussian:    (4 pi/V) sum_k exp(-k^2/4eta^2)/k^2 cos(k.r).
    The Ewald A equals this up to k_e (pi/V)(1/alpha^2 - 2/eta^2) e e^T; b is
    equal outright for a neutral electrolyte.
    """
    eta, alpha = 19.79, 2.97
    box = np.array([0.492, 0.42608, 1.5])
    rng = np.random.default_rng(7)
    elec = np.array([[0.0, 0.0, 0.0], [0.0, 0.14203, 0.0], [0.123, 0.21304, 0.0],
                     [0.123, 0.35507, 0.0], [0.246, 0.0, 0.0], [0.246, 0.14203, 0.0],
                     [0.369, 0.21304, 0.0], [0.369, 0.35507, 0.0]]).T
    sites = np.stack([rng.uniform(0, box[0], 4), rng.uniform(0, box[1], 4),
                      rng.uniform(0.3, 1.2, 4)])
    sq = np.array([0.78, -0.78, 0.5, -0.5])
    vol = box.prod()
    A = ewald.elastance(elec, box, eta, alpha, 2.0, 33.0)
    k, k2 = _all_k(box, 150.0)
    ph = k @ elec
    Ab = KE * 4 * math.pi / vol * (
        (np.cos(ph) * (np.exp(-k2 / (2 * eta * eta)) / k2)[:, None]).T @ np.cos(ph)
        + (np.sin(ph) * (np.exp(-k2 / (2 * eta * eta)) / k2)[:, None]).T @ np.sin(ph))
    const = KE * math.pi / vol * (1 / alpha ** 2 - 2 / eta ** 2)
    assert np.abs(A - Ab - const).max() < 1e-10 * np.abs(A).max()

    b = ewald.b_vector(elec, sites, sq, box, eta, alpha, 2.0, 33.0)
    k, k2 = _all_k(box, 210.0)
    bb = np.zeros(elec.shape[1])
    wk = KE * 4 * math.pi / vol * np.exp(-k2 / (4 * eta * eta)) / k2
    for i in range(elec.shape[1]):
        bb[i] = -np.sum(wk * (np.cos(k @ (elec[:, i:i + 1] - sites)) @ sq))
    assert np.abs(b - bb).max() < 1e-10 * np.abs(b).max()


# --------------------------------------------------------------------------
# P8 / P12: forces and gradient against finite differences
# --------------------------------------------------------------------------

@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_forces_match_energy_derivative(geometry):
    """F_j = -dE_cp/dR_j along q*(R) (exact Ewald, central differences, h = 1e-5 nm).

    Finite field: E_cp = U_coul - dpsi d.q + dpsi/Lz (z.q + sum Q_j Z_j);
    doubled cell: E_cp = U_coul - dpsi d.q.  A slip in either branch (a sign,
    a dropped field term) moves the derivative away from the force."""
    w, A, S = built("tiny", geometry)
    es = cpm.Electrostatics(w, "exact")
    r = cpm.step(w, A, S, es)
    h = 1e-5
    fmax = np.abs(r["f"]).max()
    for j in (0, 17, 63, w.n_site - 1):
        for d in range(3):
            xp = w.site_xyz.copy(); xp[d, j] += h
            xm = w.site_xyz.copy(); xm[d, j] -= h
            ep = cpm.step(w, A, S, es, site_xyz=xp, with_forces=False)["e_cp"]
            em = cpm.step(w, A, S, es, site_xyz=xm, with_forces=False)["e_cp"]
            assert abs(-(ep - em) / (2 * h) - r["f"][d, j]) < 1e-7 * fmax


def test_internal_forces_sum_to_zero():
    """Electrolyte-only Coulomb forces (no electrode charge) conserve momentum."""
    w = workload("tiny", "ff")
    f = ewald.coulomb_forces(w.site_xyz, w.site_q, w.elec_xyz, np.zeros(w.n_elec), w.box, w.eta,
                             w.alpha_exact, w.rcut_exact, w.kcut_exact)
    assert np.abs(f.sum(axis=1)).max() < 1e-10 * np.abs(f).max()


@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_gradient_matches_finite_differences(geometry):
    """d/dR and d/ddpsi of L = sum (q - t)^2 + U_coul by the adjoint (exact Ewald)."""
    w, A, S = built("tiny", geometry)
    es = cpm.Electrostatics(w, "exact")
    t = np.random.default_rng(5).normal(0.0, 0.01, w.n_elec)
    g = cpm.loss_gradient(w, A, S, es, t)

    def loss(x, dv):
        r = cpm.step(w, A, S, es, site_xyz=x, dv=dv, with_forces=False)
        return np.sum((r["q"] - t) ** 2) + r["u_coul"]

    h = 1e-5
    gmax = np.abs(g["dl_dx"]).max()
    for j in (3, 50, w.n_site - 9):
        for d in range(3):
            xp = w.site_xyz.copy(); xp[d, j] += h
            xm = w.site_xyz.copy(); xm[d, j] -= h
            fd = (loss(xp, w.dv) - loss(xm, w.dv)) / (2 * h)
            assert abs(fd - g["dl_dx"][d, j]) < 1e-7 * gmax
    fd = (loss(w.site_xyz, w.dv + 1e-4) - loss(w.site_xyz, w.dv - 1e-4)) / 2e-4
    assert abs(fd - g["dl_ddv"]) < 1e-8 * max(1.0, abs(fd))


# --------------------------------------------------------------------------
# P10: textbook lattice
# --------------------------------------------------------------------------

def test_rocksalt_madelung_constant():
    """Point-charge Ewald energy of rock salt gives the Madelung constant 1.747565."""
    a = 0.5628
    frac_na = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
    frac_cl = [(.5, 0, 0), (0, .5, 0), (0, 0, .5), (.5, .5, .5)]
    xyz = np.array(frac_na + frac_cl).T * a
    q = np.array([1.0] * 4 + [-1.0] * 4)
    box = np.array([a, a, a])
    u = ewald.electrolyte_energy(xyz, q, box, 6.0, 0.95, 70.0)
    madelung = -u / 4 * (a / 2) / KE
    assert abs(madelung - 1.747564594633) < 1e-9
    f = ewald.coulomb_forces(xyz, q, np.zeros((3, 0)), np.zeros(0), box, 19.79, 6.0, 0.95, 70.0)
    assert np.abs(f).max() < 1e-9


# --------------------------------------------------------------------------
# PPPM pins
# --------------------------------------------------------------------------

def test_bspline_values_and_partition():
    # M_5 at the integers: 1/24, 11/24, 11/24, 1/24 (Eulerian numbers / 4!)
    assert np.allclose(pppm.bspline(5, np.array([1.0, 2.0, 3.0, 4.0])),
                       np.array([1, 11, 11, 1]) / 24.0, atol=1e-15, rtol=0)
    u = np.random.default_rng(1).uniform(0, 30, 200)
    for P in (2, 3, 4, 5, 6, 7):
        m0 = np.floor(u - P / 2.0) + 1
        w = np.stack([pppm.bspline(P, u - (m0 + t) + P / 2.0) for t in range(P)])
        assert np.abs(w.sum(0) - 1).max() < 1e-14
        # first moment reproduces the position (B-splines are symmetric)
        assert np.abs((w * (m0 + np.arange(P)[:, None])).sum(0) - u).max() < 1e-12


def test_spread_moments_and_constant_interpolation():
    w = workload("paper", "ff")
    rho = pppm.spread(w.site_xyz, w.site_q, w.box, w.mesh, w.order)
    assert abs(rho.sum() - w.site_q.sum()) < 1e-12
    qabs = np.abs(w.site_q)
    rho_abs = pppm.spread(w.site_xyz, qabs, w.box, w.mesh, w.order)
    assert abs(rho_abs.sum() - qabs.sum()) < 1e-10
    vals = pppm.interpolate(w.elec_xyz, np.full(w.mesh, 2.5), w.box, w.order)
    assert np.abs(vals - 2.5).max() < 1e-13


def test_influence_continuum_limit():
    """At small k the optimal G is the continuum kernel deconvolved by the assignment.

    Aliases contribute O((kh/2pi)^2P) there, so G(k) U^2(k) -> 4 pi exp(-k^2/4alpha^2)/k^2
    with U(k) = prod_d sinc(k_d h_d / 2)^P.
    """
    box = np.array([3.4, 3.4, 12.625])
    mesh = (32, 32, 128)
    h = box / np.array(mesh)
    G = pppm.influence(box, mesh, 5, 2.21)
    ns, ks = pppm.mesh_wavevectors(box, mesh)
    for ix, iy, iz in ((1, 0, 0), (0, 2, 1), (1, 1, 3)):
        k = np.array([ks[0][ix], ks[1][iy], ks[2][iz]])
        k2 = k @ k
        ref = 4 * math.pi * math.exp(-k2 / (4 * 2.21 ** 2)) / k2
        x = k * h / 2
        u2 = np.prod(np.where(x == 0, 1.0, np.sin(x) / np.where(x == 0, 1.0, x)) ** 10)
        assert abs(G[ix, iy, iz] * u2 / ref - 1) < 1e-10
    # even in k (real-valued potentials)
    Gm = G[(-np.arange(mesh[0])) % mesh[0]][:, (-np.arange(mesh[1])) % mesh[1]][:, :, (-np.arange(mesh[2])) % mesh[2]]
    assert np.abs(G - Gm).max() < 1e-14 * np.abs(G).max()


def test_pppm_against_exact_ewald():
    """Discretisation budget: PPPM (order 5, h ~ 0.1 nm) against converged Ewald."""
    w, A, S = built("tiny", "ff")
    r1 = cpm.step(w, A, S, cpm.Electrostatics(w, "exact"))
    r2 = cpm.step(w, A, S, cpm.Electrostatics(w, "pppm"))
    assert np.abs(r1["q"] - r2["q"]).max() < 2e-5
    frms = np.sqrt(np.mean((r1["f"] - r2["f"]) ** 2))
    assert frms / (KE / 0.01) < 1e-5
    assert abs(r1["u_coul"] - r2["u_coul"]) < 1e-3 * abs(r1["u_coul"])


# converged Ewald parameters for the accuracy checks of the working meshes:
# erfc(alpha rc) and exp(-kc^2/4alpha^2) are both ~1e-8 (alpha rc = kc/2alpha = 4.16)
REF_ALPHA, REF_RCUT, REF_KCUT = 1.6, 2.6, 13.4


@pytest.mark.slow
@pytest.mark.parametrize("name,geometry", [("paper", "ff"), ("paper", "dc"), ("large", "ff")])
def test_working_mesh_meets_force_accuracy(name, geometry):
    """The meshes the GPU path runs (paper cell 18x18x64, doubled 18x18x128,
    large cell 36x36x64; order 5, alpha = 2.21/nm, rc = 1.2 nm) meet the
    relative force accuracy 1e-5: RMS force error against converged Ewald,
    at the same electrode charges, divided by the force between two unit
    charges 0.1 nm apart (k_e / 0.01 nm^2 = 144 eV/nm).  The charge error of
    the PPPM b against the converged b is ~1e-5 e (the discretisation budget),
    which is why the GPU's 1e-6 e bar is taken against the PPPM oracle."""
    w, A, S = built(name, geometry)
    r = cpm.step(w, A, S, cpm.Electrostatics(w, "pppm"))
    f_ref = ewald.coulomb_forces(w.site_xyz, w.site_q, w.elec_xyz, r["q"], w.box, w.eta,
                                 REF_ALPHA, REF_RCUT, REF_KCUT) + cpm.field_force(w, w.dv)
    frms = np.sqrt(np.mean((f_ref - r["f"]) ** 2)) / (KE / 0.01)
    assert frms < 1e-5
    b_ref = ewald.b_vector(w.elec_xyz, w.site_xyz, w.site_q, w.box, w.eta, REF_ALPHA, REF_RCUT, REF_KCUT)
    q_ref = S @ (b_ref + w.dv * cpm.drive_vector(w))
    assert np.abs(q_ref - r["q"]).max() < 1e-4


def test_pppm_converges_to_ewald_on_fine_mesh():
    w, A, S = built("tiny", "ff")
    wf = dataclasses.replace(w, mesh=(48, 40, 192), order=7, rcut=2.0)
    b_mesh = cpm.Electrostatics(wf, "pppm").b(w.site_xyz)
    b_exact = cpm.Electrostatics(w, "exact").b(w.site_xyz)
    d = b_mesh - b_exact
    assert np.abs(d - d.mean()).max() < 1e-8 * np.abs(b_exact - b_exact.mean()).max()


# --------------------------------------------------------------------------
# cell binning reference
# --------------------------------------------------------------------------

def test_cell_binning_is_a_valid_stable_partition():
    w = workload("paper", "dc")
    cid, start, order = cells.bin_sites(w.site_xyz, w.box, w.rcut)
    n = cells.cell_grid(w.box, w.rcut)
    assert start[-1] == w.n_site and np.all(np.diff(start) >= 0)
    for c in range(n[0] * n[1] * n[2]):
        members = order[start[c]:start[c + 1]]
        assert np.all(np.diff(members) > 0)
        assert np.all(cid[members] == c)
    # every site lies inside the box of its cell
    cz, rem = np.divmod(cid, n[0] * n[1])
    cy, cx = np.divmod(rem, n[0])
    for d, cc in enumerate((cx, cy, cz)):
        x = w.site_xyz[d] % w.box[d]
        lo = cc * w.box[d] / n[d]
        hi = (cc + 1) * w.box[d] / n[d]
        assert np.all(x >= lo - 1e-12) and np.all(x < hi + 1e-12)


def test_cell_stencil_holds_every_pair_within_the_cutoff():
    """Brute force over the site pairs of the doubled paper cell: the cells of
    two sites within rcut lie within the grid's reach of each other along
    every axis (periodically), so the stencils of the pair kernels see them."""
    w = workload("paper", "dc")
    n = cells.cell_grid(w.box, w.rcut)
    reach = cells.cell_reach(w.box, w.rcut)
    assert n[2] * w.rcut / 2 <= w.box[2] and all(
        L / m * r >= w.rcut - 1e-12 for L, m, r in zip(w.box, n, reach) if m >= 2 * r + 1)
    x = np.asarray(w.site_xyz)
    cid = cells.cell_of(x, w.box, n)
    cz, rem = np.divmod(cid, n[0] * n[1])
    cy, cx = np.divmod(rem, n[0])
    cc = (cx, cy, cz)
    d = x[:, :, None] - x[:, None, :]
    box = np.asarray(w.box)[:, None, None]
    d -= box * np.round(d / box)
    i, j = np.nonzero(((d ** 2).sum(0) < w.rcut ** 2) & ~np.eye(x.shape[1], dtype=bool))
    assert i.size > 100000
    for a in range(3):
        if n[a] >= 2 * reach[a] + 1:
            gap = np.abs(cc[a][i] - cc[a][j])
            gap = np.minimum(gap, n[a] - gap)
            assert gap.max() <= reach[a]


# --------------------------------------------------------------------------
# three charged sheets per electrode (snapshot re-solves)
# --------------------------------------------------------------------------

def test_three_layer_nearest_sheet_share():
    """With all three sheets of each electrode charged, more than 90% of each
    electrode's net charge sits on the sheet nearest the electrolyte
    (Electrolyte and Charge Densities); the next sheet carries a small charge
    of the opposite sign (the Gaussian smearing of the nearest sheet lets a
    little of the field through), and the sheets stay neutral in sum with
    their counter-electrode (e.q* = 0)."""
    from workloads import make_workload
    w = make_workload("tiny", "ff", layers=3)
    A, S = cpm.build(w)
    q = cpm.step(w, A, S, cpm.Electrostatics(w, "ewald"), dv=2.0, with_forces=False)["q"]
    assert abs(q.sum()) < 1e-12
    for side in (-1, 1):
        m = w.elec_side == side
        tot = q[m].sum()
        share = [q[m & (w.elec_layer == k)].sum() / tot for k in range(3)]
        assert share[0] > 0.9
        assert share[1] < 0 and abs(share[1]) < 0.1
        assert abs(share[2]) < abs(share[1])


def _layer_lattice_potential(dxy, dz, cx, cy, eta, nmax=40):
    """Potential (V per e on each atom of the lattice, k_e included) at a
    Gaussian charge from a rectangular cx x cy lattice of Gaussian charges of
    one basis site, offset in-plane by dxy and vertically by dz from it.

    Written from the 2D Fourier series of the interaction erf(beta r)/r,
    beta = eta/sqrt2 (two Gaussians of Eq. 2), of a lattice with cell area a:
      (2 pi k_e / a) { -[dz erf(beta dz) + exp(-beta^2 dz^2)/(beta sqrt(pi))]
        + sum_{G != 0} cos(G.dxy) [e^{G dz} erfc(G/2beta + beta dz)
                                   + e^{-G dz} erfc(G/2beta - beta dz)] / (2G) }
    (the G = 0 term up to a constant that cancels for a neutral system).  The
    self-interaction of a Gaussian is the dxy = dz = 0 term of its own lattice."""
    from scipy.special import erf, erfc
    beta = eta / math.sqrt(2.0)
    i, j = np.meshgrid(np.arange(-nmax, nmax + 1), np.arange(-nmax, nmax + 1), indexing="ij")
    G = np.stack([2 * math.pi * i / cx, 2 * math.pi * j / cy], -1).reshape(-1, 2)
    g = np.linalg.norm(G, axis=1)
    keep = g > 0
    G, g = G[keep], g[keep]
    z = abs(dz)
    # e^{Gz} erfc(G/2b + b z) written as erfcx-stable products
    t1 = np.exp(g * z - (g / (2 * beta) + beta * z) ** 2) * _erfcx(g / (2 * beta) + beta * z)
    t2 = np.exp(-g * z) * erfc(g / (2 * beta) - beta * z)
    s = np.sum(np.cos(G @ np.asarray(dxy)) * (t1 + t2) / (2 * g))
    g0 = -(z * erf(beta * z) + math.exp(-(beta * z) ** 2) / (beta * math.sqrt(math.pi)))
    return 2 * math.pi * KE / (cx * cy) * (g0 + s)


def _erfcx(x):
    from scipy.special import erfcx
    return erfcx(x)


def test_three_layer_empty_capacitor_lattice_sums():
    """Empty capacitor with three charged sheets per electrode (A-B-A), doubled
    cell with a wide back region: the charge of every atom class (sheet,
    basis site) from a small linear system built on 2D lattice sums (each
    class's potential equals its electrode's potential, total charge zero),
    against the oracle's 3D Ewald solve.  The A-B stacking makes the atoms of
    a B sheet inequivalent (above an atom or a hexagon centre of the next
    sheet), so each of the 4 basis sites of a sheet is its own class."""
    from workloads import make_workload
    w0 = make_workload("tiny", "dc", layers=3)
    n1 = w0.n_elec // 2                             # first sub-cell
    lz = 10.0                                       # back regions of ~4.3 nm
    ex = w0.elec_xyz.copy()
    ex[2, n1:] = w0.elec_xyz[2, :n1] + lz           # second sub-cell one period up
    w = dataclasses.replace(w0, box=np.array([w0.box[0], w0.box[1], 2 * lz]), elec_xyz=ex).empty()
    A, S = cpm.build(w)
    dv = 2.0
    q = S @ (dv * cpm.drive_vector(w))
    cx, cy = w.box[0] / 6, w.box[1] / 3
    # classes of the first sub-cell: atoms are generated sheet by sheet, cell
    # by cell, 4 basis sites per cell
    idx = np.arange(n1)
    per_sheet = 6 * 3 * 4
    sheet = idx // per_sheet
    basis = idx % 4
    first = {}
    for k in range(n1):
        first.setdefault((sheet[k], basis[k]), k)
    classes = sorted(first)
    nc = len(classes)
    M = np.zeros((nc + 1, nc + 1))
    rhs = np.zeros(nc + 1)
    for r, (sk, ak) in enumerate(classes):
        i = first[(sk, ak)]
        for c, (sm, bm) in enumerate(classes):
            j = first[(sm, bm)]
            M[r, c] = _layer_lattice_potential(ex[:2, i] - ex[:2, j], ex[2, i] - ex[2, j], cx, cy, w.eta)
        M[r, nc] = -1.0                             # minus the common offset psibar
        rhs[r] = dv * 0.5 * w.elec_side[i]
    M[nc, :nc] = 1.0                                # neutral
    sol = np.linalg.solve(M, rhs)
    for c, key in enumerate(classes):
        members = [k for k in range(n1) if (sheet[k], basis[k]) == key]
        assert np.abs(q[members] - sol[c]).max() < 1e-10 * np.abs(sol[:nc]).max()


# --------------------------------------------------------------------------
# slab geometry with the charged-sheet (dipole) correction
# --------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def slab_built(factor=3.0, empty=False):
    from workloads import make_workload
    w = make_workload("tiny", "slab", slab_factor=factor)
    if empty:
        w = w.empty()
    A, S = cpm.build(w)
    return w, A, S


def test_slab_empty_capacitor_closed_form():
    """The corrected slab is an isolated capacitor in z, like each sub-cell of
    the doubled cell: Q+ = eps0 A dpsi / (g - s_eff), every atom of a layer equal."""
    w, A, S = slab_built(3.0, True)
    seff = honeycomb_seff(w.box[0] / 6, w.box[1] / 3, w.eta)
    g = 4.34
    q = S @ (2.0 * cpm.drive_vector(w))
    up = w.elec_side > 0
    qdc = EPS0 * w.box[0] * w.box[1] * 2.0 / (g - seff)
    assert abs(q[up].sum() - qdc) < 1e-10 * qdc
    assert abs(q[~up].sum() + qdc) < 1e-10 * qdc
    assert np.ptp(q[up]) < 1e-12 * qdc


def test_slab_result_independent_of_the_empty_space():
    """With the correction the charges, forces and energies do not depend on
    how much empty space is added (without it they would, through the
    spurious dipole interaction of the copies)."""
    res = []
    for factor in (3.0, 4.5):
        w, A, S = slab_built(factor)
        res.append(cpm.step(w, A, S, cpm.Electrostatics(w, "exact")))
    r1, r2 = res
    assert np.abs(r1["q"] - r2["q"]).max() < 1e-10
    assert np.abs(r1["f"] - r2["f"]).max() < 1e-9 * np.abs(r1["f"]).max()
    assert abs(r1["u_coul"] - r2["u_coul"]) < 1e-10 * abs(r1["u_coul"])
    assert abs(r1["e_cp"] - r2["e_cp"]) < 1e-10 * abs(r1["e_cp"])
    # and the uncorrected sums would not be: the correction's share of q is large
    w, A, S = slab_built(3.0)
    es = cpm.Electrostatics(w, "exact")
    b_raw = es._b(w.site_xyz)
    A_raw = A - slab.elastance_term(w.elec_xyz, w.box)
    q_raw = cpm.projected_inverse(A_raw) @ (b_raw + w.dv * cpm.drive_vector(w))
    assert np.abs(q_raw - r1["q"]).max() > 1e-3 * np.abs(r1["q"]).max()


def test_slab_forces_match_energy_derivative():
    """F_j = -dE_cp/dR_j with E_cp = U_coul - dpsi d.q and the correction in U_coul."""
    w, A, S = slab_built(3.0)
    es = cpm.Electrostatics(w, "exact")
    r = cpm.step(w, A, S, es)
    h = 1e-5
    fmax = np.abs(r["f"]).max()
    for j in (2, 40, 77):
        for d in range(3):
            xp = w.site_xyz.copy(); xp[d, j] += h
            xm = w.site_xyz.copy(); xm[d, j] -= h
            ep = cpm.step(w, A, S, es, site_xyz=xp, with_forces=False)["e_cp"]
            em = cpm.step(w, A, S, es, site_xyz=xm, with_forces=False)["e_cp"]
            assert abs(-(ep - em) / (2 * h) - r["f"][d, j]) < 1e-7 * fmax


def test_slab_agrees_with_doubled_cell():
    """Filled cell: the slab and the first sub-cell of the doubled cell are both
    isolated capacitors in z, so their net electrode charges agree to rounding;
    atom by atom they differ only by the small in-plane coupling of the
    doubled cell's two electrolytes through the electrodes (~1e-4)."""
    w, A, S = slab_built(3.0)
    wd, Ad, Sd = built("tiny", "dc")
    n = w.n_elec
    up = w.elec_side > 0
    for dv in (0.0, 2.0):
        qs = cpm.step(w, A, S, cpm.Electrostatics(w, "exact"), dv=dv, with_forces=False)["q"]
        qd = cpm.step(wd, Ad, Sd, cpm.Electrostatics(wd, "exact"), dv=dv, with_forces=False)["q"][:n]
        for m in (up, ~up):
            assert abs(qs[m].sum() / qd[m].sum() - 1.0) < 1e-10
        assert np.abs(qs - qd).max() < 2e-4 * np.abs(qs).max()


# --------------------------------------------------------------------------
# 1D Poisson potential profile (Eq. 16)
# --------------------------------------------------------------------------

def _gaussian_sheets_potential(z, zs, sig, eta):
    """Isolated potential of Gaussian sheets (areal charges sig at heights zs,
    profile sig eta/sqrt(pi) exp(-eta^2 (z - zs)^2)), up to a constant:
    -(sig / 2 eps0) [u erf(eta u) + exp(-eta^2 u^2)/(eta sqrt(pi))], u = z - zs."""
    from scipy.special import erf
    out = np.zeros_like(z)
    for c, s in zip(zs, sig):
        u = z - c
        out += -(s / (2 * EPS0)) * (u * erf(eta * u) + np.exp(-(eta * u) ** 2) / (eta * math.sqrt(math.pi)))
    return out


def _charged_layers(geometry, n_bins):
    """Empty tiny capacitor (slab or doubled cell) with its closed-form charges."""
    from workloads import make_workload
    w = make_workload("tiny", geometry).empty()
    seff = honeycomb_seff(w.box[0] / 6, w.box[1] / 3, w.eta)
    area = w.box[0] * w.box[1]
    qplus = EPS0 * area * 2.0 / (4.34 - seff)
    # per-atom charge: each layer shares its electrode's net charge equally
    q = np.zeros(w.n_elec)
    for m in np.unique(np.round(w.elec_xyz[2], 9)):
        sel = np.isclose(w.elec_xyz[2], m)
        side = w.elec_side[sel][0]
        q[sel] = side * qplus / sel.sum()
    return w, q, area


@pytest.mark.parametrize("geometry", ["slab", "dc"])
def test_profile_of_gaussian_sheets(geometry):
    """Electrode Gaussians alone: the finite-difference profile converges to the
    closed-form potential of Gaussian sheets at second order in the grid step,
    and its drop between the electrode planes is (sigma/eps0)(g - 1/(eta sqrt(pi)))."""
    from oracle import profile
    errs = []
    for n_bins in (2000, 4000):
        w, q, area = _charged_layers(geometry, n_bins)
        z0 = w.elec_xyz[2].min()                     # lower electrode plane
        rho = profile.density(w, np.zeros((1, 3, 0)), q[None, :], n_bins)
        bulk = (z0 + 1.5, z0 + 2.8)
        psi = profile.potential(rho, w.box, geometry, 2.0, bulk)
        zc = (np.arange(n_bins) + 0.5) * w.box[2] / n_bins
        zs = np.unique(np.round(w.elec_xyz[2], 9))
        sig = np.array([q[np.isclose(w.elec_xyz[2], c)].sum() / area for c in zs])
        # images one period away (doubled cell: the stack is periodic)
        zz, ss = list(zs), list(sig)
        if geometry == "dc":
            for img in (-1, 1):
                zz += list(zs + img * w.box[2])
                ss += list(sig)
        exact = _gaussian_sheets_potential(zc, np.array(zz), np.array(ss), w.eta)
        sel = (zc >= bulk[0]) & (zc < bulk[1])
        exact -= exact[sel].mean()
        errs.append(np.abs(psi - exact).max())
    assert errs[0] < 2e-4 * 2.0
    assert 3.5 < errs[0] / errs[1] < 4.5              # second order
    # drop across the capacitor at the electrode planes (fine grid)
    sig_up = sig[np.argmax(sig)]
    g = 4.34
    i_lo = np.argmin(np.abs(zc - z0))
    i_hi = np.argmin(np.abs(zc - (z0 + g)))
    drop = psi[i_hi] - psi[i_lo]
    want = sig_up / EPS0 * (g - 1.0 / (w.eta * math.sqrt(math.pi)))
    assert abs(drop - want) < 2e-3 * want


def test_profile_of_point_sheets_is_exact():
    """Electrolyte charges at bin centres are sheets at grid points, and the
    second-difference solution of sheets is the piecewise-linear potential
    exactly: zero-flux ends (slab), then a finite-field rise of dpsi."""
    from oracle import profile
    from workloads import make_workload
    n_bins = 600
    w = make_workload("tiny", "slab").empty()
    h = w.box[2] / n_bins
    area = w.box[0] * w.box[1]
    zq = np.array([100.5, 250.5, 251.5, 400.5]) * h
    qq = np.array([0.7, -1.1, 0.9, -0.5])
    w = dataclasses.replace(w, site_q=qq)
    x = np.zeros((1, 3, 4))
    x[0, 2] = zq
    rho = profile.density(w, x, np.zeros((1, w.n_elec)), n_bins)
    zc = (np.arange(n_bins) + 0.5) * h
    bulk = (zc[300], zc[320])
    psi = profile.potential(rho, w.box, "slab", 0.0, bulk)
    exact = np.zeros(n_bins)
    for c, s in zip(zq, qq / area):
        exact += -(s / (2 * EPS0)) * np.abs(zc - c)
    # zero field at the ends: the point sheets are neutral, so the isolated
    # potential is flat outside them already
    sel = (zc >= bulk[0]) & (zc < bulk[1])
    exact -= exact[sel].mean()
    assert np.abs(psi - exact).max() < 1e-9 * np.abs(exact).max()
    # finite field: the same charges plus the linear rise dv z / Lz
    dv = 1.3
    wf = dataclasses.replace(w, geometry="ff")
    psi_f = profile.potential(rho, wf.box, "ff", dv, bulk)
    # a linear term solves the Laplace equation, so the solution is the
    # isolated one plus a ramp a z whose total rise over the period is dv:
    # iso(Lz) - iso(0) = p/eps0 (p the areal dipole), a Lz = dv - p/eps0
    dip = np.sum(qq / area * zq)
    ramp = (dv - dip / EPS0) * zc / w.box[2]
    ex_f = exact + ramp
    ex_f -= ex_f[sel].mean()
    assert np.abs(psi_f - ex_f).max() < 1e-9 * np.abs(ex_f).max()


# --------------------------------------------------------------------------
# the MD loop (velocity Verlet, SHAKE/RATTLE, Nose-Hoover, charges every k steps)
# --------------------------------------------------------------------------

def test_md_verlet_harmonic_closed_form():
    """Velocity Verlet on x'' = -w^2 x from rest: x_n = cos(n theta) exactly,
    cos(theta) = 1 - (w dt)^2 / 2 (the Stormer recursion)."""
    from oracle import md
    m, k, dt = np.array([2.0]), 50.0, 0.01
    w = math.sqrt(k / m[0])
    theta = math.acos(1.0 - 0.5 * (w * dt) ** 2)
    con = md.Constraints(np.zeros(0, int), np.zeros(0, int), np.zeros(0))
    box = np.array([1e6, 1e6, 1e6])
    force = lambda x: -k * x
    x = np.array([[1.0], [0.0], [0.0]])
    v = np.zeros((3, 1))
    f = force(x)
    for n in range(1, 1001):
        x, v, f = md.verlet_step(x, v, f, m, con, box, dt, force)
        assert abs(x[0, 0] - math.cos(n * theta)) < 1e-11


def test_md_rigid_rotor_constraints_and_momenta():
    """A free rigid three-site molecule: SHAKE/RATTLE keep the two bonds and
    the third side to tolerance, and momentum and angular momentum (the
    constraint forces are central pair forces) are conserved."""
    from oracle import md
    from workloads.cells import BOND, CATION_MASS
    m = np.array(CATION_MASS)
    con = md.rigid_constraints(np.array([3]), BOND)
    box = np.array([50.0, 50.0, 50.0])
    u = np.array([1.0, 0.0, 0.0]); p = np.array([0.0, 1.0, 0.0])
    c = np.array([5.0, 5.0, 5.0])
    x = np.stack([c, c + BOND * u, c + BOND * (math.cos(2 * math.pi / 3) * u + math.sin(2 * math.pi / 3) * p)], 1)
    v = md.rattle(np.random.default_rng(3).normal(0.0, 2.0, (3, 3)), x, m, con, box)
    force = lambda x: np.zeros_like(x)
    f = force(x)

    def moments(x, v):
        P = (m * v).sum(1)
        L = np.cross(x.T, (m * v).T).sum(0)
        return P, L

    P0, L0 = moments(x, v)
    for _ in range(2000):
        x, v, f = md.verlet_step(x, v, f, m, con, box, 0.002, force)
    for i, j, d in zip(con.i, con.j, con.d):
        assert abs(np.linalg.norm(x[:, i] - x[:, j]) - d) < 1e-11
        assert abs((v[:, i] - v[:, j]) @ (x[:, i] - x[:, j])) < 1e-9
    P1, L1 = moments(x, v)
    assert np.abs(P1 - P0).max() < 1e-10 * np.abs(P0).max()
    assert np.abs(L1 - L0).max() < 1e-9 * np.abs(L0).max()


@pytest.mark.slow
def test_md_extended_energy_second_order():
    """With the charges solved every step, the forces are -grad(E_cp + U_LJ),
    so the thermostatted loop conserves its extended energy up to the
    integrator's O(dt^2) error: over the same 40 fs the largest excursion of
    the extended energy shrinks about fourfold when dt is halved."""
    from oracle import md
    from workloads import md_setup
    w, A, S = built("tiny", "ff")
    base = md_setup(w)
    v0 = np.random.default_rng(8).normal(0.0, 1.0, (3, w.n_site)) * np.sqrt(md.KB * 400.0 / base.site_mass)
    excursion = []
    for dt, n in ((0.002, 20), (0.001, 40)):
        setup = dataclasses.replace(base, dt=dt, charge_every=1)
        loop = md.Loop(w, A, S, "ewald", setup, w.dv)
        s = loop.start(w.site_xyz, v0)
        h0 = loop.extended_energy(s, s.e_cp)
        hs = []
        for _ in range(n):
            s = loop.step(s)
            hs.append(loop.extended_energy(s, s.e_cp) - h0)
        excursion.append(np.abs(hs).max())
        # constraints hold along the way
        for i, j, d in zip(loop.con.i, loop.con.j, loop.con.d):
            r = md.min_image((s.x[:, i] - s.x[:, j])[:, None], w.box)[:, 0]
            assert abs(np.linalg.norm(r) - d) < 1e-10
    assert 3.0 < excursion[0] / excursion[1] < 5.5


def test_md_charges_held_between_updates():
    """Charges change only on every k-th step (k = 5), and then equal a fresh
    solve at the new positions."""
    from oracle import md
    from workloads import md_setup
    w, A, S = built("tiny", "ff")
    loop = md.Loop(w, A, S, "ewald", md_setup(w), w.dv)
    s = loop.start(w.site_xyz, np.zeros((3, w.n_site)))
    qs, xs = [s.q.copy()], [s.x.copy()]
    for _ in range(6):
        s = loop.step(s)
        qs.append(s.q.copy())
        xs.append(s.x.copy())
    for n in (1, 2, 3, 4):
        assert np.array_equal(qs[n], qs[0])
    assert not np.array_equal(qs[5], qs[4])
    fresh = cpm.step(w, A, S, cpm.Electrostatics(w, "ewald"), site_xyz=xs[5], with_forces=False)["q"]
    assert np.abs(qs[5] - fresh).max() < 1e-15
    assert np.array_equal(qs[6], qs[5])
