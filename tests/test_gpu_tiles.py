"""Batched path on the cell-tile pair kernels, in the configurations that
take their less common branches, against the oracle and the single-frame
path (one wavefront per target):

  * sites crowded into one slab: a cell holds more targets than one tile
    chunk (64) and a stencil more candidates than two LDS passes (2 x 256);
  * the tiny cell run with PPPM: cells narrower than 2 rcut, so every pair
    test loops over periodic images;
  * a batch large enough for the frames-per-launch tuner, whose frames land
    in several launches.

Bars: charges within 1e-6 e, forces within 1e-4 relative RMS of the oracle;
batched and single-frame GPU results within rounding of each other.
"""

import dataclasses
import sys

import numpy as np
import pytest

from conftest import built
from oracle import cells, cpm

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


def stencil_candidates(w, xyz):
    """(largest cell population, largest number of stencil candidates) of a frame."""
    cid, start, order = cells.bin_sites(xyz, w.box, w.rcut)
    nc = np.array(cells.cell_grid(w.box, w.rcut))
    counts = np.diff(start)
    best = 0
    for c in range(int(np.prod(nc))):
        cx, cy, cz = c % nc[0], (c // nc[0]) % nc[1], c // (nc[0] * nc[1])
        nb = set()
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    nb.add((((cz + dz) % nc[2]) * nc[1] + (cy + dy) % nc[1]) * nc[0] + (cx + dx) % nc[0])
        best = max(best, int(sum(counts[k] for k in nb)))
    return int(counts.max()), best


def run_batch_case(torch, w, A, S, frames, dvs, oracle_samples):
    from paper_2201_12963_amd import Context
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    # every frame against the single-frame path
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
    # sampled (frame, dV) pairs against the oracle
    es = cpm.Electrostatics(w, "pppm")
    for fi, vi in oracle_samples:
        ref = cpm.step(w, A, S, es, site_xyz=frames[fi], dv=dvs[vi])
        qerr = np.abs(Qb[fi, vi] - ref["q"]).max()
        fr = rel_rms(Fb[fi, vi], ref["f"])
        _say(f"    frame {fi} dV {dvs[vi]}: q err {qerr:.2e} e, F rel rms {fr:.2e}")
        assert qerr < Q_TOL
        assert fr < F_RTOL
        assert fr < 1e-9
        assert abs(Eb[fi, vi, 0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"])
        assert abs(Eb[fi, vi, 1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"])
    ctx.close()


def test_batch_tiles_with_crowded_cells(torch_dev):
    _say("[gpu] batch tiles: paper ff, sites crowded into one slab, 3 frames")
    w, A, S = built("paper", "ff")
    rng = np.random.default_rng(21)
    x = np.empty_like(w.site_xyz)
    x[0] = rng.uniform(0.0, w.box[0], w.n_site)
    x[1] = rng.uniform(0.0, w.box[1], w.n_site)
    x[2] = rng.uniform(6.2, 6.4, w.n_site)
    wc = dataclasses.replace(w, site_xyz=x)
    frames = np.stack([x, (x + rng.normal(0.0, 0.01, x.shape)) % w.box[:, None],
                       (x + rng.normal(0.0, 0.01, x.shape)) % w.box[:, None]])
    most_targets, most_candidates = stencil_candidates(wc, frames[0])
    assert most_targets > 64 and most_candidates > 512
    run_batch_case(torch_dev, wc, A, S, frames, np.array([0.0, 2.0, 3.5]), ((0, 1), (2, 2)))


@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_batch_tiles_with_periodic_images(torch_dev, geometry):
    _say(f"[gpu] batch tiles: tiny {geometry} with PPPM (cells narrower than 2 rcut), 4 frames")
    w0, A, S = built("tiny", geometry)
    w = dataclasses.replace(w0, kspace="pppm")
    assert w.rcut > 0.5 * min(w.box[0], w.box[1])
    from workloads import perturbed_frames
    frames = perturbed_frames(w, 4, sigma=0.05, seed=8)
    run_batch_case(torch_dev, w, A, S, frames, np.array([0.0, 1.0, 2.0]), ((0, 2), (3, 1)))


def test_batch_size_tuner_keeps_results(torch_dev):
    """A batch large enough to tune the frames per launch: the chosen size is
    one of the candidates, and frames that fall in different launches match
    the single-frame path."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    from paper_2201_12963_amd.binding import BUF_BATCH_CHUNK
    from workloads import perturbed_frames
    _say("[gpu] batch size tuner: paper ff, 200 frames")
    w, A, S = built("paper", "ff")
    frames = perturbed_frames(w, 200, sigma=0.05, seed=13)
    dvs = np.array([0.0, 2.0])
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    assert int(ctx.get_buffer(BUF_BATCH_CHUNK)[0]) == 0
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    tuned = ctx.get_buffer(BUF_BATCH_CHUNK)
    chunk = int(tuned[0])
    _say(f"    frames per launch {chunk}, site-pair tiles per cell {tuned[1]}, x-y planes {tuned[2]}")
    assert chunk in (64, 128)
    assert tuned[1] in (1, 2, 4) and tuned[2] in (0, 1)
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in (0, chunk - 1, chunk, 199):
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


@pytest.mark.parametrize("chunk", [4096, 2048])
def test_fp64_batch_at_full_launch_size(torch_dev, chunk, monkeypatch):
    """The FP64 batch in the launch configuration the throughput figure uses:
    4096 perturbed frames x 2 dV in launches of `chunk` frames.  Frames at
    both ends of each launch are compared with the single-frame path and two
    of them with the oracle."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    from paper_2201_12963_amd.binding import BUF_BATCH_CHUNK
    from workloads import perturbed_frames
    _say(f"[gpu] fp64 batch paper ff, 4096 frames in launches of {chunk}")
    monkeypatch.setenv("CPM_BATCH_CHUNK", str(chunk))
    w, A, S = built("paper", "ff")
    frames = perturbed_frames(w, 4096)
    dvs = np.array([0.0, 4.0])
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in (0, 2047, 2048, 4095):
        x = torch.tensor(frames[fi], dtype=torch.float64, device="cuda")
        for vi, dv in enumerate(dvs):
            with torch.cuda.stream(stream):
                q, f, e = ctx.solve(x, float(dv))
            stream.synchronize()
            q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
            assert np.abs(Qb[fi, vi] - q).max() < 1e-11
            assert rel_rms(Fb[fi, vi], f) < 1e-10
            assert np.abs(Eb[fi, vi] - e).max() < 1e-9 * np.abs(e).max()
    es = cpm.Electrostatics(w, "pppm")
    for fi, vi in ((2047, 1), (4095, 0)):
        ref = cpm.step(w, A, S, es, site_xyz=frames[fi], dv=dvs[vi])
        qerr = np.abs(Qb[fi, vi] - ref["q"]).max()
        fr = rel_rms(Fb[fi, vi], ref["f"])
        _say(f"    frame {fi} dV {dvs[vi]}: q err {qerr:.2e} e, F rel rms {fr:.2e}")
        assert qerr < 1e-8 * np.abs(ref["q"]).max() + 1e-12
        assert fr < 1e-9
        assert abs(Eb[fi, vi, 0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"])
        assert abs(Eb[fi, vi, 1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"])
    ctx.close()


def test_batch_with_planes_too_large_for_three_per_workgroup(torch_dev):
    """FP64 x-y planes of 48 x 45 points: three of them (with the ping-pong
    copies) exceed the LDS of a workgroup, so the many-frame x-y launches take
    one plane per workgroup; the batch must still match the single frames."""
    _say("[gpu] batch tiles: tiny ff with PPPM mesh 48x45x64, 3 frames")
    w0, A, S = built("tiny", "ff")
    w = dataclasses.replace(w0, kspace="pppm", mesh=(48, 45, 64))
    assert (2 * 3 * 48 * 45 + 48 + 45) * 16 > 150 * 1024
    from workloads import perturbed_frames
    frames = perturbed_frames(w, 3, sigma=0.05, seed=9)
    run_batch_case(torch_dev, w, A, S, frames, np.array([0.0, 2.0]), ((1, 1),))


def test_calls_outside_the_context_stream(torch_dev):
    """solve, solve_batch, grad and the autograd loss called on torch's current
    stream (not inside `with torch.cuda.stream(ctx.stream)`) give the same
    results as calls inside it: the binding orders the two streams."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    from paper_2201_12963_amd.autograd import cpm_loss
    from workloads import perturbed_frames
    _say("[gpu] calls outside the context stream, paper ff")
    w, A, S = built("paper", "ff")
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    frames = perturbed_frames(w, 4, sigma=0.05, seed=3)
    dvs = np.array([0.0, 2.0])
    t = torch.tensor(np.random.default_rng(2).normal(0, 0.01, w.n_elec), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        X = torch.tensor(frames, dtype=torch.float64, device="cuda")
        ref_solve = [a.clone() for a in ctx.solve(X[1].contiguous(), 2.0)]
        ref_batch = [a.clone() for a in ctx.solve_batch(X, dvs)]
        ref_grad = [a.clone() for a in ctx.grad(X[2].contiguous(), 2.0, t)]
    stream.synchronize()
    for rep in range(3):
        # inputs made on the current stream right before the call, outputs read right after
        X2 = torch.tensor(frames, dtype=torch.float64, device="cuda") * 1.0
        got = ctx.solve(X2[1].contiguous(), 2.0)
        for a, b in zip(got, ref_solve):
            assert torch.allclose(a, b, rtol=0, atol=1e-12 * float(b.abs().max()))
        got = ctx.solve_batch(X2, dvs)
        for a, b in zip(got, ref_batch):
            assert torch.allclose(a, b, rtol=0, atol=1e-12 * float(b.abs().max()))
        got = ctx.grad(X2[2].contiguous(), 2.0, t)
        for a, b in zip(got, ref_grad):
            assert torch.allclose(a, b, rtol=0, atol=1e-11 * float(b.abs().max()))
        x = X2[2].clone().requires_grad_(True)
        dv = torch.tensor(2.0, dtype=torch.float64, device="cuda", requires_grad=True)
        loss, q = cpm_loss(ctx, x, dv, t)
        loss.backward()
        assert abs(loss.item() - ref_grad[0].item()) < 1e-11 * abs(ref_grad[0].item())
        assert torch.allclose(x.grad, ref_grad[1], rtol=0, atol=1e-11 * float(ref_grad[1].abs().max()))
    ctx.close()


@pytest.mark.parametrize("tiles_per_cell,xy_planes", [(1, 1), (2, 0), (4, 1), (3, 0)])
def test_batch_launch_shapes(torch_dev, tiles_per_cell, xy_planes):
    """Every launch shape the tuner may pick (and one it does not) gives the
    single-frame results: site-pair tiles split 1-4 ways per cell, one or
    several x-y planes per workgroup."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    from workloads import perturbed_frames
    _say(f"[gpu] batch shape: {tiles_per_cell} tiles per cell, x-y planes {xy_planes}")
    w, A, S = built("paper", "dc")
    frames = perturbed_frames(w, 40, sigma=0.05, seed=19)
    dvs = np.array([0.5, 3.0])
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    ctx.set_batch_shape(16, tiles_per_cell, xy_planes)
    X = torch.tensor(frames, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(X, dvs)
    stream.synchronize()
    assert ctx.sync_status() == 0
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi in (0, 17, 39):
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
