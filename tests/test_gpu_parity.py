"""GPU path against the CPU oracle, element by element, through the C-ABI.

Bars (from the method's accuracy targets): electrode charges within 1e-6 e
per atom, forces within 1e-4 relative RMS.  FP64 stages are also held to a
rounding-level bound (1e-9 relative) to catch slips the loose bars would hide;
integer work (cell binning) is compared bit for bit.
"""

import math
import sys

import numpy as np
import pytest

from conftest import built, workload
from oracle import KE, cells, cpm, ewald, pppm

pytestmark = pytest.mark.gpu

Q_TOL = 1e-6          # e per atom
F_RTOL = 1e-4         # relative RMS
TIGHT = 1e-9          # FP64 rounding-level bound (relative)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def gpu_context(torch, w, precision=0):
    from paper_2201_12963_amd import Context
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, precision=precision, stream=stream)
    ctx.build_elastance()
    return ctx, stream


def oracle_method(w):
    return "pppm" if w.kspace == "pppm" else "ewald"


CASES = [("tiny", "ff"), ("tiny", "dc"), ("paper", "ff"), ("paper", "dc")]


@pytest.mark.parametrize("name,geometry", CASES)
def test_elastance_and_projection(torch_dev, name, geometry):
    _say(f"[gpu] elastance {name} {geometry}")
    w, A, S = built(name, geometry)
    ctx, _ = gpu_context(torch_dev, w)
    Ag = ctx.get_matrix(0)
    Sg = ctx.get_matrix(1)
    Scg = ctx.get_matrix(2)
    assert np.abs(Ag - A).max() < 1e-11 * np.abs(A).max()
    assert np.abs(Sg - S).max() < 1e-8 * np.abs(S).max()
    assert np.abs(Scg - S @ cpm.drive_vector(w)).max() < 1e-8 * np.abs(Scg).max()
    assert np.abs(Sg @ np.ones(w.n_elec)).max() < 1e-10 * np.abs(Sg).max()
    if geometry == "dc":
        assert np.abs(Sg @ w.elec_sub.astype(float)).max() < 1e-10 * np.abs(Sg).max()
    ctx.close()


@pytest.mark.parametrize("name,geometry", CASES)
def test_step_parity(torch_dev, name, geometry):
    _say(f"[gpu] step {name} {geometry}")
    w, A, S = built(name, geometry)
    check_step(torch_dev, w, A, S)


def test_step_parity_sites_crowded_into_one_layer(torch_dev):
    """All sites in a 0.2 nm slab: on the planes beside it a wavefront of the
    spread stages more sites than it has lanes (its list takes several
    rounds), the path an ordinary cell never takes."""
    import dataclasses
    _say("[gpu] step paper ff, sites crowded into one slab")
    w, A, S = built("paper", "ff")
    rng = np.random.default_rng(11)
    x = np.empty_like(w.site_xyz)
    x[0] = rng.uniform(0.0, w.box[0], w.n_site)
    x[1] = rng.uniform(0.0, w.box[1], w.n_site)
    x[2] = rng.uniform(6.2, 6.4, w.n_site)
    wc = dataclasses.replace(w, site_xyz=x)
    # sites whose z stencil reaches each plane, per staging wavefront: the
    # spread's first 256 threads read sites u * 256 + thread (u < 16), so
    # site j belongs to wavefront (j mod 256) // 64 of batch j // 4096
    u = x[2] / (w.box[2] / w.mesh[2])
    first = (np.floor(u - w.order / 2.0).astype(int) + 1) % w.mesh[2]
    j = np.arange(w.n_site)
    group = (j // 4096) * 4 + (j % 256) // 64
    per_wave = np.zeros((w.mesh[2], group.max() + 1), int)
    for t in range(w.order):
        np.add.at(per_wave, ((first + t) % w.mesh[2], group), 1)
    assert per_wave.max() > 64
    check_step(torch_dev, wc, A, S)


@pytest.mark.parametrize("kz", [600, 2048])
def test_step_parity_long_z_columns(torch_dev, kz):
    """Meshes with more points along z than the z pass prefetches per lane
    (512), and at 2048 points so long that a workgroup holds one column."""
    import dataclasses
    _say(f"[gpu] step tiny ff with PPPM, mesh 16x16x{kz}")
    w0, A, S = built("tiny", "ff")
    w = dataclasses.replace(w0, kspace="pppm", mesh=(16, 16, kz))
    check_step(torch_dev, w, A, S)


@pytest.mark.parametrize("kx,ky", [(15, 20), (30, 16), (32, 20), (25, 24)])
def test_step_parity_plane_shapes(torch_dev, kx, ky):
    """Odd and non-square x-y planes.  A one-frame step sums lines of up to 32
    points directly while every output of the plane has a thread of its own
    (15 x 20, 30 x 16); larger planes (32 x 20, 25 x 24) take the radix
    stages."""
    import dataclasses
    _say(f"[gpu] step tiny ff with PPPM, mesh {kx}x{ky}x64")
    w0, A, S = built("tiny", "ff")
    w = dataclasses.replace(w0, kspace="pppm", mesh=(kx, ky, 64))
    check_step(torch_dev, w, A, S)


@pytest.mark.parametrize("order", [3, 4, 6, 7])
def test_step_parity_spline_orders(torch_dev, order):
    """B-spline orders other than 5: the kernels evaluate the weights by the
    Cox-de Boor triangle there and by closed-form quartics at order 5."""
    import dataclasses
    _say(f"[gpu] step tiny ff with PPPM, order {order}")
    w0, A, S = built("tiny", "ff")
    w = dataclasses.replace(w0, kspace="pppm", mesh=(16, 16, 64), order=order)
    check_step(torch_dev, w, A, S)


def test_step_parity_odd_site_count(torch_dev):
    """99 sites: the one-frame site-force kernel pairs two wavefronts per
    site when all of them fit on the device, and the last workgroup then
    holds a single site (its second pair mirrors the last site and writes
    nothing)."""
    import dataclasses
    _say("[gpu] step tiny ff with PPPM, 99 sites")
    w0, A, S = built("tiny", "ff")
    q = w0.site_q[:99].copy()
    q[0] = 0.0                                   # keeps the electrolyte neutral
    w = dataclasses.replace(w0, kspace="pppm", site_xyz=w0.site_xyz[:, :99].copy(), site_q=q)
    check_step(torch_dev, w, A, S)


def check_step(torch, w, A, S):
    es = cpm.Electrostatics(w, oracle_method(w))
    ref = cpm.step(w, A, S, es)
    ctx, stream = gpu_context(torch, w)
    xyz = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        q, f, e = ctx.solve(xyz, w.dv)
    stream.synchronize()
    assert ctx.sync_status() == 0
    q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()

    # a1: cell binning, bit for bit
    cid, start, order = cells.bin_sites(w.site_xyz, w.box, w.rcut)
    assert np.array_equal(ctx.get_buffer(7), np.array(cells.cell_grid(w.box, w.rcut)))
    assert np.array_equal(ctx.get_buffer(0), start)
    assert np.array_equal(ctx.get_buffer(1), order)

    # a2: real-space electrolyte potential at the electrodes
    phir = ewald.electrolyte_potential_realspace(w.elec_xyz, w.site_xyz, w.site_q, w.box, w.eta, w.alpha, w.rcut)
    phir_g = ctx.get_buffer(2)
    assert np.abs(phir_g - phir).max() <= TIGHT * np.abs(phir).max()

    if w.kspace == "pppm":
        # a3: charge mesh; a4-a6: potential mesh
        rho = pppm.spread(w.site_xyz, w.site_q, w.box, w.mesh, w.order)
        rho_g = ctx.get_buffer(4).reshape(w.mesh[::-1]).transpose(2, 1, 0)
        assert np.abs(rho_g - rho).max() < TIGHT * np.abs(rho).max()
        phi = KE * pppm.mesh_potential(rho, es.G, w.box)
        phi_g = ctx.get_buffer(5).reshape(w.mesh[::-1]).transpose(2, 1, 0)
        assert np.abs(phi_g - phi).max() < TIGHT * np.abs(phi).max()
        # a9: field of all charges on the mesh
        rho_all = rho + pppm.spread(w.elec_xyz, q, w.box, w.mesh, w.order)
        E = KE * pppm.mesh_field(rho_all, es.G, w.box)
        E_g = ctx.get_buffer(6).reshape((3,) + tuple(w.mesh[::-1])).transpose(0, 3, 2, 1)
        assert np.abs(E_g - E).max() < TIGHT * np.abs(E).max()

    # a7: b
    b_g = ctx.get_buffer(3)
    assert np.abs(b_g - ref["b"]).max() < TIGHT * np.abs(ref["b"]).max()
    # a8: charges (spec bar and rounding-level bound)
    qerr = np.abs(q - ref["q"]).max()
    _say(f"    q max err {qerr:.3e} e, |q|max {np.abs(ref['q']).max():.3e}")
    assert qerr < Q_TOL
    assert qerr < 1e-8 * np.abs(ref["q"]).max() + 1e-12
    assert abs(q.sum()) < 1e-10
    # a9/a10: forces
    fr = rel_rms(f, ref["f"])
    _say(f"    F rel rms {fr:.3e}")
    assert fr < F_RTOL
    assert fr < 1e-9
    # a11: energies
    _say(f"    U_coul {e[0]:.12f} vs {ref['u_coul']:.12f}; E_cp {e[1]:.12f} vs {ref['e_cp']:.12f}")
    assert abs(e[0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"]) + 1e-9
    assert abs(e[1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"]) + 1e-9
    ctx.close()


def test_graph_replay_matches_eager(torch_dev):
    """A context created with the graph flag replays its captured step (several
    times, with eager work between) and agrees with a context that launches
    directly, to rounding (the charge spread adds with LDS atomics)."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    _say("[gpu] graph replay paper ff")
    w, A, S = built("paper", "ff")
    stream = torch.cuda.Stream()
    ctx_e = Context.from_workload(w, stream=stream)
    ctx_e.build_elastance()
    ctx_g = Context.from_workload(w, stream=stream, graph=True)
    ctx_g.set_matrix(ctx_e.get_matrix(1))
    xyz = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        ref = ctx_e.solve(xyz, w.dv)
    stream.synchronize()
    q0 = torch.empty(w.n_elec, dtype=torch.float64, device="cuda")
    f0 = torch.empty((3, w.n_site), dtype=torch.float64, device="cuda")
    e0 = torch.empty(2, dtype=torch.float64, device="cuda")
    for it in range(4):
        with torch.cuda.stream(stream):
            q0.zero_(); f0.zero_(); e0.zero_()
            ctx_g.solve(xyz, w.dv, q0, f0, e0)
            junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
        stream.synchronize()
        for got, want in zip((q0, f0, e0), ref):
            assert torch.allclose(got, want, rtol=0, atol=1e-12 * float(want.abs().max()))
    ctx_e.close()
    ctx_g.close()


def test_set_matrix_restores_a_built_context(torch_dev):
    """A context given S from a host copy (checkpoint resume) steps like the one that built it.

    Equal to rounding, not bit for bit: the charge spread adds with LDS
    atomics, whose order varies from run to run."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    _say("[gpu] set_matrix paper dc")
    w, A, S = built("paper", "dc")
    ctx1, stream = gpu_context(torch, w)
    ctx2 = Context.from_workload(w, stream=stream)
    ctx2.set_matrix(ctx1.get_matrix(1))
    xyz = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        r1 = ctx1.solve(xyz, w.dv)
        r2 = ctx2.solve(xyz, w.dv)
    stream.synchronize()
    for a, b in zip(r1, r2):
        assert torch.allclose(a, b, rtol=0, atol=1e-12 * float(b.abs().max()))
    ctx1.close()
    ctx2.close()


def test_nonfinite_positions_are_reported(torch_dev):
    torch = torch_dev
    w, A, S = built("tiny", "ff")
    ctx, stream = gpu_context(torch, w)
    x = w.site_xyz.copy()
    x[0, 3] = np.nan
    xyz = torch.tensor(x, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        ctx.solve(xyz, w.dv)
    stream.synchronize()
    assert ctx.sync_status() == -6
    assert ctx.sync_status() == 0
    ctx.close()


def test_solve_before_build_is_a_state_error(torch_dev):
    torch = torch_dev
    from paper_2201_12963_amd import Context, CpmError
    w = workload("tiny", "ff")
    ctx = Context.from_workload(w, stream=torch.cuda.Stream())
    xyz = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    with pytest.raises(CpmError) as ei:
        ctx.solve(xyz, 2.0)
    assert ei.value.code == -2
    ctx.close()


def test_coincident_electrodes_are_not_positive_definite(torch_dev):
    torch = torch_dev
    import dataclasses
    from paper_2201_12963_amd import Context, CpmError
    w = workload("tiny", "ff")
    ex = w.elec_xyz.copy()
    ex[:, 1] = ex[:, 0]
    ctx = Context.from_workload(dataclasses.replace(w, elec_xyz=ex), stream=torch.cuda.Stream())
    with pytest.raises(CpmError) as ei:
        ctx.build_elastance()
    assert ei.value.code == -3
    ctx.close()
