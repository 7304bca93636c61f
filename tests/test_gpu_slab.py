"""Slab geometry (z period lengthened with empty space, charged-sheet dipole
correction) on the GPU against the oracle: the setting the paper's fully
periodic methods are compared with (Fig. 2b; Computational Efficiency).

Cells: the tiny cell with explicit Ewald and with PPPM (period 18 nm, mesh
16 x 16 x 192), and the paper-shaped cell with PPPM (period 37.875 nm, mesh
18 x 18 x 192, the finite-field mesh's spacing), one frame, the adjoint
gradient and a batch.
"""

import functools
import sys

import numpy as np
import pytest

from oracle import KE, cpm, ewald, pppm

pytestmark = pytest.mark.gpu

Q_TOL = 1e-6
F_RTOL = 1e-4
TIGHT = 1e-9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@functools.lru_cache(maxsize=None)
def slab_case(name, kspace):
    import dataclasses
    from workloads import make_workload
    w = make_workload(name, "slab")
    if kspace != w.kspace:
        w = dataclasses.replace(w, kspace=kspace)
    A, S = cpm.build(w)
    return w, A, S


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def make_ctx(torch, w):
    from paper_2201_12963_amd import Context
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    return ctx, stream


@pytest.mark.parametrize("name,kspace", [("tiny", "ewald"), ("tiny", "pppm"), ("paper", "pppm")])
def test_slab_step_parity(torch_dev, name, kspace):
    torch = torch_dev
    _say(f"[gpu] slab {name} {kspace}")
    w, A, S = slab_case(name, kspace)
    es = cpm.Electrostatics(w, kspace)
    ref = cpm.step(w, A, S, es)
    ctx, stream = make_ctx(torch, w)
    Ag = ctx.get_matrix(0)
    assert np.abs(Ag - A).max() < 1e-11 * np.abs(A).max()
    assert np.abs(ctx.get_matrix(1) - S).max() < 1e-8 * np.abs(S).max()
    with torch.cuda.stream(stream):
        q, f, e = ctx.solve(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv)
    stream.synchronize()
    assert ctx.sync_status() == 0
    q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
    b_g = ctx.get_buffer(3)
    assert np.abs(b_g - ref["b"]).max() < TIGHT * np.abs(ref["b"]).max()
    qerr = np.abs(q - ref["q"]).max()
    fr = rel_rms(f, ref["f"])
    _say(f"    q err {qerr:.2e} e, F rel rms {fr:.2e}, U_coul {e[0]:.10f} vs {ref['u_coul']:.10f}")
    assert qerr < Q_TOL
    assert qerr < 1e-8 * np.abs(ref["q"]).max() + 1e-12
    assert fr < 1e-9
    assert abs(e[0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"])
    assert abs(e[1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"])
    ctx.close()


def test_slab_gradient_parity(torch_dev):
    torch = torch_dev
    _say("[gpu] slab gradient paper pppm")
    w, A, S = slab_case("paper", "pppm")
    es = cpm.Electrostatics(w, "pppm")
    t = np.random.default_rng(4).normal(0.0, 0.01, w.n_elec)
    ref = cpm.loss_gradient(w, A, S, es, t)
    ctx, stream = make_ctx(torch, w)
    with torch.cuda.stream(stream):
        loss, dldx, dldv, q = ctx.grad(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv,
                                       torch.tensor(t, dtype=torch.float64, device="cuda"))
    stream.synchronize()
    assert abs(loss.item() - ref["loss"]) < 1e-9 * abs(ref["loss"])
    assert rel_rms(dldx.cpu().numpy(), ref["dl_dx"]) < 1e-9
    assert abs(dldv.item() - ref["dl_ddv"]) < 1e-8 * abs(ref["dl_ddv"]) + 1e-12
    ctx.close()


def test_slab_batch(torch_dev):
    torch = torch_dev
    from workloads import perturbed_frames
    _say("[gpu] slab batch paper pppm, 96 frames")
    w, A, S = slab_case("paper", "pppm")
    # perturb inside the cell only (the empty space must stay empty)
    frames = perturbed_frames(w, 96, sigma=0.05, seed=12)
    frames[:, 2, :] = np.clip(frames[:, 2, :], w.site_zmin, w.site_zmax)
    dvs = np.array([0.0, 1.0, 2.5])
    ctx, stream = make_ctx(torch, w)
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(torch.tensor(frames, dtype=torch.float64, device="cuda"), dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in (0, 95):
        x = torch.tensor(frames[fi], dtype=torch.float64, device="cuda")
        for vi, dv in enumerate(dvs):
            with torch.cuda.stream(stream):
                q, f, e = ctx.solve(x, float(dv))
            stream.synchronize()
            assert np.abs(Qb[fi, vi] - q.cpu().numpy()).max() < 1e-11
            assert rel_rms(Fb[fi, vi], f.cpu().numpy()) < 1e-10
            assert np.abs(Eb[fi, vi] - e.cpu().numpy()).max() < 1e-9 * np.abs(e.cpu().numpy()).max()
    es = cpm.Electrostatics(w, "pppm")
    ref = cpm.step(w, A, S, es, site_xyz=frames[40], dv=dvs[2])
    assert np.abs(Qb[40, 2] - ref["q"]).max() < Q_TOL
    assert rel_rms(Fb[40, 2], ref["f"]) < 1e-9
    assert abs(Eb[40, 2, 1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"])
    ctx.close()
