"""The allocation-free variant of the profile call (cpm_profile_noalloc)
against the allocating one (cpm_profile), through the C-ABI, on two calls
in a row, the second with fewer frames and bins.  Bars: charge density to
1e-11 relative (the histograms add with LDS atomics in any order), potential
to 1e-9 relative."""

import ctypes
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


def test_profile_noalloc_matches_profile(torch_dev):
    torch = torch_dev
    from paper_2201_12963_amd import Context
    from paper_2201_12963_amd.binding import load_library
    from workloads import make_workload, perturbed_frames
    lib = load_library()
    fn = lib.cpm_profile_noalloc
    vp, ip = ctypes.c_void_p, ctypes.c_int
    fn.argtypes = [vp, ip, vp, vp, ctypes.c_longlong, ctypes.c_double, ip, ctypes.c_double, ctypes.c_double, vp, vp]
    fn.restype = ip
    w = make_workload("paper", "dc")
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    frames = perturbed_frames(w, 300, sigma=0.05, seed=31)
    frames[:, 2, :] = np.clip(frames[:, 2, :], w.site_zmin, w.site_zmax)
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    dvs = np.array([0.0, 2.0])
    with torch.cuda.stream(stream):
        Q, _, _ = ctx.solve_batch(X, dvs, forces=False, energy=False)
    stream.synchronize()
    bulk = (5.0, 8.0)
    for n_frames, n_bins in ((300, 1600), (40, 700)):
        _say(f"[gpu] profile noalloc vs profile: paper dc, {n_frames} frames, {n_bins} bins")
        Xs = X[:n_frames]
        Qs = Q[:n_frames, 1]
        with torch.cuda.stream(stream):
            rho_a, psi_a = ctx.profile(Xs, Qs, 2.0, n_bins, bulk)
            rho_b = torch.empty(n_bins, dtype=torch.float64, device="cuda")
            psi_b = torch.empty(n_bins, dtype=torch.float64, device="cuda")
            r = fn(ctx._ctx, n_frames, ctypes.c_void_p(Xs.data_ptr()), ctypes.c_void_p(Qs.data_ptr()),
                   Qs.stride(0), 2.0, n_bins, bulk[0], bulk[1], ctypes.c_void_p(rho_b.data_ptr()),
                   ctypes.c_void_p(psi_b.data_ptr()))
        assert r == 0, lib.cpm_last_error(ctx._ctx)
        stream.synchronize()
        assert ctx.sync_status() == 0
        ra, rb = rho_a.cpu().numpy(), rho_b.cpu().numpy()
        pa, pb = psi_a.cpu().numpy(), psi_b.cpu().numpy()
        _say(f"    rho {np.abs(ra - rb).max() / np.abs(ra).max():.2e}, psi {np.abs(pa - pb).max() / np.abs(pa).max():.2e}")
        assert np.abs(ra - rb).max() < 1e-11 * np.abs(ra).max()
        assert np.abs(pa - pb).max() < 1e-9 * np.abs(pa).max()
    ctx.close()
