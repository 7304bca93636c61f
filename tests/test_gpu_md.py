"""The constant-potential MD loop on the GPU against the oracle's loop.

Both start from the same positions and seeded velocities, integrate the same
number of 2 fs steps (velocity Verlet, Nose-Hoover, SHAKE/RATTLE, Lennard-Jones,
charges re-solved every fifth step) and are compared step for step: the
per-step kinetic and Lennard-Jones energies, and at the end positions,
velocities, charges and the thermostat variables.  Cases: the paper-shaped
cell in finite field (rigid 3-site cations, PPPM) and doubled cell (two
thermostats), and the tiny cell with explicit Ewald (single-site ions, a
0.6 nm Lennard-Jones cutoff that its 1.278 nm side allows).
"""

import sys

import numpy as np
import pytest

from conftest import built

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,geometry,n_steps", [("paper", "ff", 11), ("paper", "dc", 11), ("tiny", "ff", 11)])
def test_md_loop_parity(torch_dev, name, geometry, n_steps):
    torch = torch_dev
    from oracle import md
    from paper_2201_12963_amd import Context, MDLoop
    from workloads import md_setup
    _say(f"[gpu] md loop {name} {geometry}, {n_steps} steps")
    import dataclasses
    w, A, S = built(name, geometry)
    setup = md_setup(w)
    if name == "tiny":      # its 1.278 nm side holds a minimum-image cutoff of at most 0.639 nm
        setup = dataclasses.replace(setup, lj_cut=0.6)
    v0 = np.random.default_rng(17).normal(0.0, 1.0, (3, w.n_site)) * np.sqrt(md.KB * setup.temperature /
                                                                             setup.site_mass)
    method = "pppm" if w.kspace == "pppm" else "ewald"
    loop = md.Loop(w, A, S, method, setup, w.dv)
    s = loop.start(w.site_xyz, v0)
    ke_ref, ulj_ref = [], []
    for _ in range(n_steps):
        s = loop.step(s)
        ke_ref.append(loop.kinetic(s))
        ulj_ref.append(s.u_lj)
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    mdl = MDLoop(ctx, setup)
    x = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    v = torch.tensor(v0, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        q, th = mdl.run(x, v, w.dv, 6)
        q, th2 = mdl.run(x, v, w.dv, n_steps - 6)          # a second call continues the loop
    stream.synchronize()
    assert ctx.sync_status() == 0
    th = np.concatenate([th.cpu().numpy(), th2.cpu().numpy()])
    xg, vg, qg = x.cpu().numpy(), v.cpu().numpy(), q.cpu().numpy()
    xi, eta, step = mdl.state()
    dx = np.abs(xg - s.x).max()
    dvel = np.abs(vg - s.v).max() / np.abs(s.v).max()
    dq = np.abs(qg - s.q).max()
    _say(f"    x {dx:.2e} nm, v rel {dvel:.2e}, q {dq:.2e} e, xi {np.abs(xi - s.xi).max():.2e}, "
         f"KE rel {np.abs(th[:, 0] - ke_ref).max() / max(ke_ref):.2e}")
    assert step == n_steps
    assert dx < 1e-9
    assert dvel < 1e-8
    assert dq < 1e-9
    assert np.abs(xi - s.xi).max() < 1e-8 * max(1.0, np.abs(s.xi).max())
    assert np.abs(eta - s.eta).max() < 1e-10 * max(1.0, np.abs(s.eta).max())
    assert np.abs(th[:, 0] - ke_ref).max() < 1e-8 * max(ke_ref)
    assert np.abs(th[:, 1] - ulj_ref).max() < 1e-8 * max(1.0, np.abs(ulj_ref).max())
    # constraints hold on the GPU trajectory
    for i, j, d in zip(loop.con.i, loop.con.j, loop.con.d):
        r = md.min_image((xg[:, i] - xg[:, j])[:, None], w.box)[:, 0]
        assert abs(np.linalg.norm(r) - d) < 1e-10
    mdl.close()
    ctx.close()


@pytest.mark.parametrize("graph", [False, True])
def test_md_loop_after_another_solve_on_the_context(torch_dev, graph):
    """Between charge updates the loop reuses the electrode charge's x-y
    spectrum (PPPM) and sorted charges of the last update.  A solve of other
    positions on the same context in between replaces the sorted charges;
    the loop must notice and rebuild them from its own charges, so that the
    trajectory is the one without the interruption.  With graph capture on,
    the second solve is a replay of the first one's graph, which runs none of
    the host-side enqueue code."""
    torch = torch_dev
    from oracle import md
    from paper_2201_12963_amd import Context, MDLoop
    from workloads import md_setup, perturbed_frames
    _say(f"[gpu] md loop paper ff (PPPM), solves between runs, graph={graph}")
    w, A, S = built("paper", "ff")
    setup = md_setup(w)
    v0 = np.random.default_rng(23).normal(0.0, 1.0, (3, w.n_site)) * np.sqrt(md.KB * setup.temperature /
                                                                             setup.site_mass)
    other = perturbed_frames(w, 1, sigma=0.2, seed=5)[0]
    results = []
    for interrupt in (False, True):
        stream = torch.cuda.Stream()
        ctx = Context.from_workload(w, stream=stream, graph=graph)
        ctx.build_elastance()
        mdl = MDLoop(ctx, setup)
        x = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
        v = torch.tensor(v0, dtype=torch.float64, device="cuda")
        xo = torch.tensor(other, dtype=torch.float64, device="cuda")
        qo = torch.empty(w.n_elec, dtype=torch.float64, device="cuda")
        fo = torch.empty((3, w.n_site), dtype=torch.float64, device="cuda")
        eo = torch.empty(2, dtype=torch.float64, device="cuda")
        with torch.cuda.stream(stream):
            mdl.run(x, v, w.dv, 7)                   # ends two steps after an update
            if interrupt:
                ctx.solve(xo, 0.5 * w.dv, qo, fo, eo)
            mdl.run(x, v, w.dv, 6)                   # ends three steps after an update
            if interrupt:
                ctx.solve(xo, 0.5 * w.dv, qo, fo, eo)   # the same arguments (graph: a replay)
            q, _ = mdl.run(x, v, w.dv, 6)
        stream.synchronize()
        assert ctx.sync_status() == 0
        results.append((x.cpu().numpy(), v.cpu().numpy(), q.cpu().numpy()))
        mdl.close()
        ctx.close()
    (xa, va, qa), (xb, vb, qb) = results
    _say(f"    x {np.abs(xa - xb).max():.2e} nm, v {np.abs(va - vb).max():.2e}, q {np.abs(qa - qb).max():.2e} e")
    assert np.abs(xa - xb).max() < 1e-11
    assert np.abs(va - vb).max() < 1e-8 * np.abs(va).max()
    assert np.abs(qa - qb).max() < 1e-11
