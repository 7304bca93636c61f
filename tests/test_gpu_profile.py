"""Charge density and 1D Poisson potential profile (Eq. 16) on the GPU,
through the C-ABI, against the oracle's histogram and finite-difference
matrix solve on the same frames and charges.

Cases: the paper-shaped cell in finite field (400 bins, the paper's grid of
~0.034 nm per cell), doubled cell (800) and slab (1200), frames and charges
from a GPU batch (one dV of the batch read through its stride), three-sheet
electrodes, and 4096 frames (the most histogram partitions) at 2048 bins.
"""

import sys

import numpy as np
import pytest

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


def bulk_window(w):
    """Middle of the electrolyte: the paper averages 100 grid points there."""
    zlo, zhi = w.site_zmin.min(), w.site_zmax.max()
    mid = 0.5 * (zlo + zhi)
    return (mid - 1.7, mid + 1.7)


def run_case(torch, w, n_frames, n_bins, dvs, v):
    from oracle import profile
    from paper_2201_12963_amd import Context
    from workloads import perturbed_frames
    frames = perturbed_frames(w, n_frames, sigma=0.05, seed=21)
    frames[:, 2, :] = np.clip(frames[:, 2, :], w.site_zmin, w.site_zmax)
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    bulk = bulk_window(w)
    with torch.cuda.stream(stream):
        Q, _, _ = ctx.solve_batch(X, dvs, forces=False, energy=False)
        rho, psi = ctx.profile(X, Q[:, v], float(dvs[v]), n_bins, bulk)
    stream.synchronize()
    assert ctx.sync_status() == 0
    rho, psi = rho.cpu().numpy(), psi.cpu().numpy()
    q = Q[:, v].cpu().numpy()
    rho_ref = profile.density(w, frames, q, n_bins)
    psi_ref = profile.potential(rho_ref, w.box, w.geometry, float(dvs[v]), bulk)
    drho = np.abs(rho - rho_ref).max() / np.abs(rho_ref).max()
    dpsi = np.abs(psi - psi_ref).max() / np.abs(psi_ref).max()
    _say(f"    rho rel err {drho:.2e}, psi rel err {dpsi:.2e}, |psi| max {np.abs(psi_ref).max():.3f} V")
    assert drho < 1e-11
    assert dpsi < 1e-9
    ctx.close()
    return rho, psi


@pytest.mark.parametrize("geometry,n_bins", [("ff", 400), ("dc", 800), ("slab", 1200)])
def test_profile_parity(torch_dev, geometry, n_bins):
    from workloads import make_workload
    _say(f"[gpu] profile paper {geometry}, 24 frames, {n_bins} bins")
    w = make_workload("paper", geometry)
    run_case(torch_dev, w, 24, n_bins, np.array([0.0, 2.5]), 1)


def test_profile_three_sheet_electrodes(torch_dev):
    from workloads import make_workload
    _say("[gpu] profile paper ff, three charged sheets, 8 frames, 400 bins")
    w = make_workload("paper", "ff", layers=3)
    run_case(torch_dev, w, 8, 400, np.array([2.0]), 0)


def test_profile_many_frames_most_partitions(torch_dev):
    from workloads import make_workload
    _say("[gpu] profile paper ff, 4096 frames, 2048 bins")
    w = make_workload("paper", "ff")
    run_case(torch_dev, w, 4096, 2048, np.array([0.0, 1.0]), 1)


def test_profile_rejects_bad_arguments(torch_dev):
    torch = torch_dev
    from paper_2201_12963_amd import Context, CpmError
    from workloads import make_workload
    w = make_workload("tiny", "ff")
    ctx = Context.from_workload(w, stream=torch.cuda.Stream())
    X = torch.tensor(w.site_xyz[None], dtype=torch.float64, device="cuda")
    q = torch.zeros((1, w.n_elec), dtype=torch.float64, device="cuda")
    for n_bins, bulk in ((1, (1.0, 2.0)), (4096, (1.0, 2.0)), (100, (2.0, 2.0))):
        with pytest.raises(CpmError) as ei:
            ctx.profile(X, q, 0.0, n_bins, bulk)
        assert ei.value.code == -1
    ctx.close()
