"""Three-layer electrodes (all graphene sheets charged) on the GPU.

The paper charges only the sheet of each electrode nearest the electrolyte
during production and re-solves saved snapshots with all three sheets
charged, finding that more than 90% of the induced charge stays on the
nearest sheet (Electrolyte and Charge Densities; appendix, post-analysis).
Here the same re-solve runs through the C-ABI on the paper-shaped cell
(2640 charged atoms in the finite field, 5280 in the doubled cell), one
frame and batched, against the oracle.
"""

import functools
import sys

import numpy as np
import pytest

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


@functools.lru_cache(maxsize=None)
def built3(name, geometry):
    from workloads import make_workload
    w = make_workload(name, geometry, layers=3)
    A, S = cpm.build(w)
    return w, A, S


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def proximal_fraction(w, q):
    """Net charge of the nearest sheets over the net charge of the electrodes,
    per electrode (and, in the doubled cell, per sub-cell)."""
    out = []
    subs = (w.elec_sub == 1, w.elec_sub == 0) if w.geometry == "dc" else (np.ones(w.n_elec, bool),)
    for sub in subs:
        for side in (-1, 1):
            m = sub & (w.elec_side == side)
            out.append(q[..., m & (w.elec_layer == 0)].sum(-1) / q[..., m].sum(-1))
    return np.array(out)


@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_three_layer_step_and_batch(torch_dev, geometry):
    torch = torch_dev
    from paper_2201_12963_amd import Context
    from workloads import perturbed_frames
    _say(f"[gpu] three-layer paper {geometry}")
    w, A, S = built3("paper", geometry)
    es = cpm.Electrostatics(w, "pppm")
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    assert np.abs(ctx.get_matrix(1) - S).max() < 1e-8 * np.abs(S).max()
    ref = cpm.step(w, A, S, es)
    with torch.cuda.stream(stream):
        q, f, e = ctx.solve(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv)
    stream.synchronize()
    q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
    _say(f"    one frame: q err {np.abs(q - ref['q']).max():.2e} e, F rel rms {rel_rms(f, ref['f']):.2e}")
    assert np.abs(q - ref["q"]).max() < Q_TOL
    assert rel_rms(f, ref["f"]) < 1e-9
    assert abs(e[0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"])
    assert abs(e[1] - ref["e_cp"]) < 1e-9 * abs(ref["e_cp"])
    # batched re-solve of snapshots over a dV sweep (63 frames: the last group
    # of frames that share the electrode spread's staging is a partial one)
    frames = perturbed_frames(w, 63, sigma=0.05, seed=6)
    dvs = np.array([0.0, 1.2, 2.5])
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(torch.tensor(frames, dtype=torch.float64, device="cuda"), dvs)
    stream.synchronize()
    Qb, Fb, Eb = Qb.cpu().numpy(), Fb.cpu().numpy(), Eb.cpu().numpy()
    for fi, vi in ((0, 2), (62, 1)):
        r = cpm.step(w, A, S, es, site_xyz=frames[fi], dv=dvs[vi])
        qerr = np.abs(Qb[fi, vi] - r["q"]).max()
        _say(f"    frame {fi} dV {dvs[vi]}: q err {qerr:.2e} e, F rel rms {rel_rms(Fb[fi, vi], r['f']):.2e}")
        assert qerr < Q_TOL
        assert rel_rms(Fb[fi, vi], r["f"]) < 1e-9
        assert abs(Eb[fi, vi, 0] - r["u_coul"]) < 1e-9 * abs(r["u_coul"])
    # the paper's observation on the re-solved snapshots at 2.5 V
    frac = proximal_fraction(w, Qb[:, 2])
    _say(f"    nearest-sheet share of the electrode charge at 2.5 V: min {frac.min():.4f}, "
         f"mean {frac.mean():.4f}")
    assert frac.min() > 0.9
    ctx.close()


@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_three_layer_mixed_single_frame(torch_dev, geometry):
    """The precision form on 2640 (5280 in the doubled cell) charged atoms
    against the oracle, one frame and a batch of 7 (whose electrode spread
    stages 4, or 2, frames per workgroup, the last group a partial one);
    more than 4096 atoms need no special path."""
    torch = torch_dev
    from paper_2201_12963_amd import Context, MIXED
    from workloads import perturbed_frames
    _say(f"[gpu] three-layer paper {geometry}, mixed precision")
    w, A, S = built3("paper", geometry)
    es = cpm.Electrostatics(w, "pppm")
    ref = cpm.step(w, A, S, es)
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, precision=MIXED, stream=stream)
    ctx.build_elastance()
    with torch.cuda.stream(stream):
        q, f, e = ctx.solve(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv)
    stream.synchronize()
    q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
    dq = np.abs(q - ref["q"]).max()
    _say(f"    mixed vs oracle: q max {dq:.3e} e, F rel rms {rel_rms(f, ref['f']):.3e}, "
         f"U_coul {abs(e[0] - ref['u_coul']):.3e} eV")
    assert dq < Q_TOL
    assert rel_rms(f, ref["f"]) < F_RTOL
    assert abs(q.sum()) < 1e-12
    if geometry == "dc":
        assert abs(q[w.elec_sub == 1].sum()) < 1e-12
    frames = perturbed_frames(w, 7, sigma=0.05, seed=8)
    dvs = np.array([0.0, 2.5])
    with torch.cuda.stream(stream):
        Qb, Fb, Eb = ctx.solve_batch(torch.tensor(frames, dtype=torch.float64, device="cuda"), dvs)
    stream.synchronize()
    r = cpm.step(w, A, S, es, site_xyz=frames[6], dv=dvs[1])
    qb, fb = Qb[6, 1].cpu().numpy(), Fb[6, 1].cpu().numpy()
    _say(f"    mixed batch frame 6 dV {dvs[1]}: q max {np.abs(qb - r['q']).max():.3e} e, "
         f"F rel rms {rel_rms(fb, r['f']):.3e}")
    assert np.abs(qb - r["q"]).max() < Q_TOL
    assert rel_rms(fb, r["f"]) < F_RTOL
    ctx.close()
