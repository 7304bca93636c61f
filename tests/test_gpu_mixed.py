"""Mixed-precision form and full-size cells on the GPU.

The mixed path (FP32 mesh, FFT and real space, FP32 GEMV on centred b or the
bf16x3 split GEMM for batches, FP64 re-projection and energy sums) is
compared per result (charges, forces, U_coul, E_cp) with the FP64 oracle on
the same inputs and held to the method's bars (1e-6 e per charge, 1e-4
relative RMS force); its distance from the FP64 GPU path is printed beside
it.  The FP64 path at the largest cell (6.8 x 6.8 nm, 3520 electrode atoms,
5120 sites) is compared with the oracle.
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


def solve_both(torch, w, frames=None, dvs=None):
    from paper_2201_12963_amd import Context, FP64, MIXED
    out = {}
    for prec in (FP64, MIXED):
        stream = torch.cuda.Stream()
        ctx = Context.from_workload(w, precision=prec, stream=stream)
        ctx.build_elastance()
        with torch.cuda.stream(stream):
            if frames is None:
                r = ctx.solve(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv)
            else:
                r = ctx.solve_batch(torch.tensor(frames, dtype=torch.float64, device="cuda"), dvs)
        stream.synchronize()
        out[prec] = tuple(t.cpu().numpy() for t in r)
        ctx.close()
    return out[FP64], out[MIXED]


@pytest.mark.parametrize("name,geometry", [("paper", "ff"), ("paper", "dc"), ("large", "ff")])
def test_mixed_single_frame(torch_dev, name, geometry):
    _say(f"[gpu] mixed {name} {geometry}")
    w, A, S = built(name, geometry)
    ref = cpm.step(w, A, S, cpm.Electrostatics(w, "pppm"))
    (q64, f64, e64), (q32, f32, e32) = solve_both(torch_dev, w)
    dq = np.abs(q32 - ref["q"]).max()
    df = rel_rms(f32, ref["f"])
    du = abs(e32[0] - ref["u_coul"])
    de = abs(e32[1] - ref["e_cp"])
    _say(f"    mixed vs oracle: q max {dq:.3e} e (|q| max {np.abs(ref['q']).max():.3e}), F rel rms {df:.3e}, "
         f"U_coul {du:.3e} eV of {abs(ref['u_coul']):.3e}, E_cp {de:.3e} eV")
    _say(f"    mixed vs fp64 GPU: q max {np.abs(q32 - q64).max():.3e} e, F rel rms {rel_rms(f32, f64):.3e}")
    assert dq < Q_TOL
    assert df < F_RTOL
    assert abs(q32.sum()) < 1e-12
    assert du < 1e-5 * abs(ref["u_coul"]) + 1e-6
    assert de < 1e-5 * abs(ref["e_cp"]) + 1e-6
    if geometry == "dc":
        assert abs(q32[w.elec_sub.astype(bool)].sum()) < 1e-12


@pytest.mark.parametrize("geometry", ["ff", "dc"])
def test_mixed_batch(torch_dev, geometry):
    from workloads import perturbed_frames
    _say(f"[gpu] mixed batch paper {geometry}")
    w, A, S = built("paper", geometry)
    frames = perturbed_frames(w, 8, sigma=0.05, seed=4)
    dvs = np.linspace(0.0, 4.0, 5)
    (q64, f64, e64), (q32, f32, e32) = solve_both(torch_dev, w, frames, dvs)
    _say(f"    bf16x3 batch vs fp64 GPU: q max {np.abs(q32 - q64).max():.3e} e, F rel rms {rel_rms(f32, f64):.3e}")
    es = cpm.Electrostatics(w, "pppm")
    for fi, vi in ((0, 0), (3, 2), (7, 4)):
        ref = cpm.step(w, A, S, es, site_xyz=frames[fi], dv=dvs[vi])
        dq = np.abs(q32[fi, vi] - ref["q"]).max()
        df = rel_rms(f32[fi, vi], ref["f"])
        du = abs(e32[fi, vi, 0] - ref["u_coul"])
        _say(f"    frame {fi} dV {dvs[vi]}: mixed vs oracle q max {dq:.3e} e, F rel rms {df:.3e}, U_coul {du:.3e} eV")
        assert dq < Q_TOL
        assert df < F_RTOL
        assert du < 1e-5 * abs(ref["u_coul"]) + 1e-6
        assert abs(e32[fi, vi, 1] - ref["e_cp"]) < 1e-5 * abs(ref["e_cp"]) + 1e-6
    if geometry == "dc":
        sub = w.elec_sub.astype(bool)
        assert np.abs(q32[..., sub].sum(-1)).max() < 1e-12


def test_large_cell_fp64_against_oracle(torch_dev):
    """Full size of the precision and gradient workloads (3520 electrode atoms, 5120 sites)."""
    torch = torch_dev
    from paper_2201_12963_amd import Context
    _say("[gpu] large ff fp64 vs oracle (oracle build takes a while)")
    w, A, S = built("large", "ff")
    es = cpm.Electrostatics(w, "pppm")
    ref = cpm.step(w, A, S, es)
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, stream=stream)
    ctx.build_elastance()
    assert np.abs(ctx.get_matrix(1) - S).max() < 1e-8 * np.abs(S).max()
    with torch.cuda.stream(stream):
        q, f, e = ctx.solve(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv)
    stream.synchronize()
    q, f, e = q.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
    _say(f"    q max err {np.abs(q - ref['q']).max():.3e}, F rel rms {rel_rms(f, ref['f']):.3e}")
    assert np.abs(q - ref["q"]).max() < Q_TOL
    assert rel_rms(f, ref["f"]) < 1e-9
    assert abs(e[0] - ref["u_coul"]) < 1e-9 * abs(ref["u_coul"])
    # the adjoint at full size against the oracle's
    t = np.random.default_rng(5).normal(0.0, 0.01, w.n_elec)
    g = cpm.loss_gradient(w, A, S, es, t)
    with torch.cuda.stream(stream):
        loss, dldx, dldv, _ = ctx.grad(torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda"), w.dv,
                                        torch.tensor(t, dtype=torch.float64, device="cuda"))
    stream.synchronize()
    assert abs(loss.item() - g["loss"]) < 1e-9 * abs(g["loss"])
    assert rel_rms(dldx.cpu().numpy(), g["dl_dx"]) < 1e-9
    assert abs(dldv.item() - g["dl_ddv"]) < 1e-8 * abs(g["dl_ddv"])
    ctx.close()


def test_mixed_batch_many_frames_within_bar(torch_dev):
    """4096 perturbed frames: every mixed-precision charge within 1e-6 e of FP64,
    and sampled frames within the bars of the oracle.

    Guards the two places where FP32 would otherwise cross the bar on a few
    frames: displacements of ~10 nm coordinates (formed in FP64) and the
    real-space cutoff test (taken in FP64, so both paths keep the same pairs)."""
    from workloads import perturbed_frames
    _say("[gpu] mixed batch, 4096 frames paper ff")
    w, A, S = built("paper", "ff")
    frames = perturbed_frames(w, 4096)
    dvs = np.array([0.0, 4.0])
    (q64, _, _), (q32, f32, e32) = solve_both(torch_dev, w, frames, dvs)
    per_frame = np.abs(q32 - q64).max(axis=(1, 2))
    _say(f"    max {per_frame.max():.3e} e, frames above 1e-6: {int((per_frame > Q_TOL).sum())}")
    assert per_frame.max() < Q_TOL
    es = cpm.Electrostatics(w, "pppm")
    for fi, vi in ((int(np.argmax(per_frame)), 1), (4095, 0)):
        ref = cpm.step(w, A, S, es, site_xyz=frames[fi], dv=dvs[vi])
        dq = np.abs(q32[fi, vi] - ref["q"]).max()
        df = rel_rms(f32[fi, vi], ref["f"])
        _say(f"    frame {fi} dV {dvs[vi]}: mixed vs oracle q max {dq:.3e} e, F rel rms {df:.3e}")
        assert dq < Q_TOL
        assert df < F_RTOL
        assert abs(e32[fi, vi, 0] - ref["u_coul"]) < 1e-5 * abs(ref["u_coul"]) + 1e-6
