"""GPU forms beyond the single step: the adjoint gradient and batched frames.

Adjoint: the GPU gradient is compared with the oracle's adjoint gradient
(same k-space method) and with central finite differences of the GPU loss.
Batch: every (frame, dV) of a batch is compared with a single-frame GPU
solve and, for sampled frames, with the oracle.
"""

import sys

import numpy as np
import pytest

from conftest import built, workload
from oracle import cpm

pytestmark = pytest.mark.gpu

Q_TOL = 1e-6
F_RTOL = 1e-4


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


@pytest.mark.parametrize("name,geometry", [("tiny", "ff"), ("tiny", "dc"), ("paper", "ff"), ("paper", "dc")])
def test_gradient_parity(torch_dev, name, geometry):
    torch = torch_dev
    _say(f"[gpu] gradient {name} {geometry}")
    w, A, S = built(name, geometry)
    es = cpm.Electrostatics(w, "pppm" if w.kspace == "pppm" else "ewald")
    t = np.random.default_rng(11).normal(0.0, 0.01, w.n_elec)
    ref = cpm.loss_gradient(w, A, S, es, t)
    ctx, stream = gpu_context(torch, w)
    xyz = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    tt = torch.tensor(t, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        loss, dldx, dldv, q = ctx.grad(xyz, w.dv, tt)
    stream.synchronize()
    loss, dldx, dldv, q = loss.item(), dldx.cpu().numpy(), dldv.item(), q.cpu().numpy()
    _say(f"    loss {loss:.12f} vs {ref['loss']:.12f}; dL/ddV {dldv:.10e} vs {ref['dl_ddv']:.10e}; "
         f"dL/dR rel rms {rel_rms(dldx, ref['dl_dx']):.3e}")
    assert np.abs(q - ref["q"]).max() < Q_TOL
    assert abs(loss - ref["loss"]) < 1e-9 * abs(ref["loss"])
    assert abs(dldv - ref["dl_ddv"]) < 1e-8 * abs(ref["dl_ddv"]) + 1e-12
    assert rel_rms(dldx, ref["dl_dx"]) < 1e-9

    # central differences of the GPU loss (h = 1e-5 nm)
    h = 1e-5
    gmax = np.abs(dldx).max()
    tol = 1e-6 if w.kspace == "ewald" else 2e-3        # PPPM ik forces are not the exact mesh gradient
    for j, d in ((5, 0), (w.n_site // 2, 2), (w.n_site - 3, 1)):
        vals = []
        for sgn in (1, -1):
            x = w.site_xyz.copy()
            x[d, j] += sgn * h
            with torch.cuda.stream(stream):
                l, *_ = ctx.grad(torch.tensor(x, dtype=torch.float64, device="cuda"), w.dv, tt)
            stream.synchronize()
            vals.append(l.item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dldx[d, j]) < tol * gmax, (j, d, fd, dldx[d, j])
    ctx.close()


def test_autograd_function(torch_dev):
    torch = torch_dev
    from paper_2201_12963_amd.autograd import cpm_loss
    w, A, S = built("tiny", "ff")
    ctx, stream = gpu_context(torch, w)
    t = torch.zeros(w.n_elec, dtype=torch.float64, device="cuda")
    x = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda", requires_grad=True)
    dv = torch.tensor(w.dv, dtype=torch.float64, device="cuda", requires_grad=True)
    with torch.cuda.stream(stream):
        loss, q = cpm_loss(ctx, x, dv, t)
        (2.0 * loss).backward()
    stream.synchronize()
    es = cpm.Electrostatics(w, "ewald")
    ref = cpm.loss_gradient(w, A, S, es, np.zeros(w.n_elec))
    assert rel_rms(x.grad.cpu().numpy(), 2.0 * ref["dl_dx"]) < 1e-9
    assert abs(dv.grad.item() - 2.0 * ref["dl_ddv"]) < 1e-8 * abs(ref["dl_ddv"])
    ctx.close()


@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_batch_matches_single_frames(torch_dev, geometry):
    torch = torch_dev
    from workloads import perturbed_frames
    _say(f"[gpu] batch paper {geometry}")
    w, A, S = built("paper", geometry)
    frames = perturbed_frames(w, 6, sigma=0.05, seed=4)
    dvs = np.array([0.0, 0.7, 2.0, 4.0])
    ctx, stream = gpu_context(torch, w)
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in range(frames.shape[0]):
        x = torch.tensor(frames[fi], dtype=torch.float64, device="cuda")
        for vi, dv in enumerate(dvs):
            with torch.cuda.stream(stream):
                q, f, e = ctx.solve(x, float(dv))
            stream.synchronize()
            q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
            assert np.abs(Qb[fi, vi] - q).max() < 1e-11
            assert rel_rms(Fb[fi, vi], f) < 1e-10
            assert np.abs(Eb[fi, vi] - e).max() < 1e-9 * np.abs(e).max()
    # sampled frames against the oracle
    es = cpm.Electrostatics(w, "pppm")
    for fi, vi in ((0, 2), (5, 3)):
        ref = cpm.step(w, A, S, es, site_xyz=frames[fi], dv=dvs[vi])
        assert np.abs(Qb[fi, vi] - ref["q"]).max() < Q_TOL
        assert rel_rms(Fb[fi, vi], ref["f"]) < F_RTOL
        assert abs(Eb[fi, vi, 0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"])
        assert abs(Eb[fi, vi, 1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"])
    ctx.close()


@pytest.mark.parametrize("order", [4, 6])
def test_batch_matches_single_frames_other_spline_orders(torch_dev, order):
    """Batches at B-spline orders other than 5: the site forces gather the
    field meshes (the per-plane interpolation inside the inverse x-y pass
    takes order 5 only), and the planes the electrode stencils reach differ
    from order 5's.  The batch is compared with single frames of the same
    context; the single-frame path at these orders is compared with the
    oracle in test_step_parity_spline_orders."""
    torch = torch_dev
    import dataclasses
    from workloads import perturbed_frames
    _say(f"[gpu] batch paper ff, order {order}")
    w0, _, _ = built("paper", "ff")
    w = dataclasses.replace(w0, order=order)
    frames = perturbed_frames(w, 5, sigma=0.05, seed=9)
    dvs = np.array([0.0, 1.5, 4.0])
    ctx, stream = gpu_context(torch, w)
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in (0, 4):
        x = torch.tensor(frames[fi], dtype=torch.float64, device="cuda")
        for vi, dv in enumerate(dvs):
            with torch.cuda.stream(stream):
                q, f, e = ctx.solve(x, float(dv))
            stream.synchronize()
            q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
            assert np.abs(Qb[fi, vi] - q).max() < 1e-11
            assert rel_rms(Fb[fi, vi], f) < 1e-10
            assert np.abs(Eb[fi, vi] - e).max() < 1e-9 * np.abs(e).max()
    ctx.close()


def test_batch_matches_single_frames_long_z_mesh(torch_dev):
    """A z mesh of more than 256 planes: the many-frame passes then transform
    the electrode charge on every plane (the field pass has no plane mask),
    while the potential still goes only to the planes the electrode stencils
    reach, and the interpolation's candidate layers span the longer mesh."""
    torch = torch_dev
    import dataclasses
    from workloads import perturbed_frames
    _say("[gpu] batch paper ff, mesh 18x18x288")
    w0, _, _ = built("paper", "ff")
    w = dataclasses.replace(w0, mesh=(18, 18, 288))
    frames = perturbed_frames(w, 4, sigma=0.05, seed=12)
    dvs = np.array([0.0, 3.0])
    ctx, stream = gpu_context(torch, w)
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in (0, 3):
        x = torch.tensor(frames[fi], dtype=torch.float64, device="cuda")
        for vi, dv in enumerate(dvs):
            with torch.cuda.stream(stream):
                q, f, e = ctx.solve(x, float(dv))
            stream.synchronize()
            q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
            assert np.abs(Qb[fi, vi] - q).max() < 1e-11
            assert rel_rms(Fb[fi, vi], f) < 1e-10
            assert np.abs(Eb[fi, vi] - e).max() < 1e-9 * np.abs(e).max()
    ctx.close()


def test_batch_matches_single_frames_large_cell(torch_dev):
    """The batched pair tiles on a grid whose x-y stencil is a proper subset of
    the cross-section (5 x 5 cells in x-y, 21 along z): forward stencils of
    several runs, periodic wraps in x and y, each pair once.  The one-frame
    path of the same cell is held to the oracle in test_gpu_mixed."""
    torch = torch_dev
    from workloads import perturbed_frames
    _say("[gpu] batch large ff")
    w = workload("large", "ff")
    frames = perturbed_frames(w, 3, sigma=0.05, seed=9)
    dvs = np.array([0.0, 3.0])
    ctx, stream = gpu_context(torch, w)
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in range(frames.shape[0]):
        x = torch.tensor(frames[fi], dtype=torch.float64, device="cuda")
        for vi, dv in enumerate(dvs):
            with torch.cuda.stream(stream):
                q, f, e = ctx.solve(x, float(dv))
            stream.synchronize()
            q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
            assert np.abs(Qb[fi, vi] - q).max() < 1e-11
            assert rel_rms(Fb[fi, vi], f) < 1e-10
            assert np.abs(Eb[fi, vi] - e).max() < 1e-9 * np.abs(e).max()
    ctx.close()
