"""Benchmark of the constant-potential electrostatics step on one MI355X.

Headline workload (paper-shaped cell): 3.4 x 3.4 nm periodic cell, proximal
graphene layers of 440 atoms per electrode, 320 coarse-grained ion pairs,
PPPM order 5 at 1e-5 force accuracy, a random-walk trajectory of
sigma = 0.005 nm per step.  A step is one pass of the whole path on one
configuration: cell binning, real-space and PPPM b, q = S b + dV S c, PPPM
field and real-space forces, energies.  The headline value is the doubled
cell (N_e = 1760, N_l = 2560); the finite-field cell (N_e = 880, N_l = 1280),
the precision form, the batched form and the gradient are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
    python bench.py --only {precision,batched,gradient}     (one form alone)

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # FP64 vector (and FP64 matrix) peak
BF16_PEAK_TFLOPS = 2500.0      # dense bf16 matrix peak
FP32_PEAK_TFLOPS = 157.3       # FP32 vector peak (the mixed form's pair arithmetic)
REPLAYS = int(os.environ.get("CPM_BENCH_REPLAYS", "200"))

# Algorithmic FP64 operation counts of the per-pair formulas (erfc ~ 20 and
# exp ~ 10 operations as polynomial/rational evaluations, plus the arithmetic
# around them): potential g1 pair 50, force g0 pair 50, force g1 pair 80.
FLOPS_PAIR_B, FLOPS_PAIR_G0, FLOPS_PAIR_G1 = 50, 50, 80


def count_pairs(a, b, box, rcut, same=False):
    """Number of (a, b) pairs within rcut (minimum image; the cells used here
    are >= 2 rcut).  same=True counts the unordered pairs of one set once."""
    n = 0
    for i0 in range(0, a.shape[1], 512):
        d = a[:, i0:i0 + 512, None] - b[:, None, :]
        d -= box[:, None, None] * np.round(d / box[:, None, None])
        r2 = np.einsum("kab,kab->ab", d, d)
        n += int(np.count_nonzero(r2 < rcut * rcut))
    if same:
        n = (n - a.shape[1]) // 2
    return n


_PAIRS = {}


def pair_counts(w):
    """(unordered site-site pairs, site-electrode pairs) within r_c, cached per workload."""
    key = (w.name, w.geometry, w.n_elec, w.n_site)
    if key not in _PAIRS:
        _PAIRS[key] = (count_pairs(w.site_xyz, w.site_xyz, w.box, w.rcut, same=True),
                       count_pairs(w.site_xyz, w.elec_xyz, w.box, w.rcut))
    return _PAIRS[key]


def listed_planes(w):
    """Number of z planes that the electrode atoms' order-P stencils reach
    (stencil of grid coordinate u from floor(u - P/2) + 1, as the library
    builds it)."""
    kz, lz, p = w.mesh[2], w.box[2], w.order
    u = np.mod(w.elec_xyz[2], lz) * (kz / lz)
    first = np.unique(np.floor(u - p / 2.0).astype(np.int64) + 1)
    return len({int((f + t) % kz) for f in first for t in range(p)})


def kernel_work(w, name, n_frames=1, n_dv=1, mixed=False):
    """(bound, algorithmic work of one launch over n_frames frames, unit) of a
    step kernel.  Bytes count frame-independent tables (S, S c, electrode
    stencils, the influence function) once per launch and per-frame data
    once per frame; FLOP counts are per frame.  Site pairs are the unordered
    pairs within r_c (each is one evaluation of the method).  In batches the
    cell tiles take the site-electrode (g1) pairs as well, and the site-force
    kernel only interpolates the mesh field."""
    P3 = w.order ** 3
    M = int(np.prod(w.mesh))
    ne, nl = w.n_elec, w.n_site
    pg0, pg1 = pair_counts(w)
    batched = n_frames > 1
    if name == "site_pairs":
        flop = pg0 * FLOPS_PAIR_G0 + (pg1 * FLOPS_PAIR_G1 if batched else 0)
        return "alu", n_frames * flop, "TFLOP/s"
    if name == "site_forces":
        flop = nl * P3 * 6 + (0 if batched else pg1 * FLOPS_PAIR_G1)
        return "alu", n_frames * flop, "TFLOP/s"
    if name == "real_b":
        return "alu", n_frames * pg1 * FLOPS_PAIR_B, "TFLOP/s"
    if name == "gemm":              # Q0 = S B: 2 N_e^2 FLOP per frame (the method's contraction)
        return "mfma" if mixed else "alu", n_frames * 2.0 * ne * ne, "TFLOP/s"
    if name == "expand_q":          # Q0 read, q written for every dV; S c once
        return "hbm", ne * 8 + n_frames * ne * 8 * (1 + n_dv), "GB/s"
    if name == "expand_f":          # two force vectors read, F written for every dV
        return "hbm", n_frames * 3 * nl * 8 * (2 + n_dv), "GB/s"
    if name == "charges":           # S streamed once; b read, Q0 and q written per frame
        return "hbm", 8 * ne * ne + n_frames * 8 * 3 * ne, "GB/s"
    # mesh passes: reals of the form's precision; in batches the electrode
    # charge's forward and the potential's inverse x-y passes, and the
    # potential's z-pass output and the field z pass's electrode input, cover
    # only the planes the electrode stencils reach (ML points)
    elt = 4 if mixed else 8
    cpx = 2 * elt
    ML = listed_planes(w) * w.mesh[0] * w.mesh[1] if batched and w.mesh[2] <= 256 else M
    if name == "fft_z_pot":         # G once; spectrum read, saved for the field pass, result written
        return "hbm", M * elt + n_frames * (M * cpx * 2 + ML * cpx), "GB/s"
    if name == "fft_z_field":       # G once; saved and electrode spectra read, two field spectra written
        return "hbm", M * elt + n_frames * (M * cpx * 3 + ML * cpx), "GB/s"
    if name == "fft_xy_fwd":        # the spread's launch: sites in, the complex planes out
        return "hbm", n_frames * (nl * 32 + M * cpx), "GB/s"
    if name in ("fft_xy_inv", "fft_xy_fwd_e"):   # real plane in, complex plane out (or back)
        return "hbm", n_frames * ML * (elt + cpx), "GB/s"
    if name == "fft_xy_inv_e":      # two field spectra in; three field meshes out (batches at
        #                             order 5: the 30 per-plane shares of every site instead)
        out = nl * 30 * elt if batched and w.order == 5 else M * 3 * elt
        return "hbm", n_frames * (M * cpx * 2 + out), "GB/s"
    if name == "spread_elec":       # stencil table once; q read, mesh written per frame
        return "hbm", ne * P3 * (4 + elt) + n_frames * (ne * 8 + ML * elt), "GB/s"
    if name == "gather_b":          # stencil table once; mesh read, b written per frame
        return "hbm", ne * P3 * (4 + elt) + n_frames * (ML * elt + ne * 16), "GB/s"
    if name == "bin":               # positions and charges in; sorted copies, order and the
        #                             wrapped-coordinate scratch (written and read back) out
        return "hbm", n_frames * nl * (32 + 36 + 48), "GB/s"
    # energy: S c, c, d, z once; Q0 and b per frame, the site energies per frame
    return "hbm", ne * 8 * 4 + n_frames * (ne * 16 + nl * 8), "GB/s"


def make_ctx(torch, w, precision=0):
    from paper_2201_12963_amd import Context
    stream = torch.cuda.Stream()
    ctx = Context.from_workload(w, precision=precision, stream=stream)
    ctx.build_elastance()
    return ctx, stream


def gpu_steps(torch, w, traj, steps, warmup, precision=0, profile_kernels=False):
    """Time `steps` steps of the trajectory (inputs resident on the GPU)."""
    ctx, stream = make_ctx(torch, w, precision)
    frames = torch.tensor(traj, dtype=torch.float64, device="cuda")
    xyz = torch.empty((3, w.n_site), dtype=torch.float64, device="cuda")
    q = torch.empty(w.n_elec, dtype=torch.float64, device="cuda")
    f = torch.empty((3, w.n_site), dtype=torch.float64, device="cuda")
    e = torch.empty(2, dtype=torch.float64, device="cuda")
    nfr = frames.shape[0]
    with torch.cuda.stream(stream):
        for k in range(warmup):
            xyz.copy_(frames[k % nfr])
            ctx.solve(xyz, w.dv, q, f, e)
    stream.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    with torch.cuda.stream(stream):
        t0.record(stream)
        for k in range(steps):
            xyz.copy_(frames[k % nfr])
            ctx.solve(xyz, w.dv, q, f, e)
        t1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    out = dict(ms_total=t0.elapsed_time(t1), wall_s=wall, q=q.cpu().numpy(), f=f.cpu().numpy(),
               e=e.cpu().numpy())
    if ctx.sync_status() != 0:
        raise RuntimeError("kernel status flag raised during the timed loop")
    if profile_kernels:
        if os.environ.get("CPM_BENCH_COPY_CALIBRATION"):
            # a plain device copy of known size (256 MiB read, 256 MiB
            # written), for scaling the HBM byte counters of a --pmc run
            src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.mul(src, 1.0, out=dst)          # the same bytes through an elementwise kernel
            torch.cuda.synchronize()
            del src, dst
        out["kernel_ms"] = kernel_times(torch, ctx, stream, REPLAYS)
    ctx.close()
    return out


def kernel_times(torch, ctx, stream, reps, warm=5):
    """Average duration (ms) of the last launch of every step kernel: each is
    replayed `reps` times, bracketed by events on the context's stream."""
    from paper_2201_12963_amd.binding import KERNELS
    times = {}
    for kid, name in enumerate(KERNELS):
        try:
            with torch.cuda.stream(stream):
                ctx.replay_kernel(kid, warm)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                ctx.replay_kernel(kid, reps)
                b.record(stream)
            stream.synchronize()
            times[name] = a.elapsed_time(b) / reps
        except Exception:
            continue
    return times


def peak_of(bound, mixed=False):
    if bound == "hbm":
        return HBM_PEAK_GBS
    if bound == "mfma":
        return BF16_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
    return FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS


def per_kernel_roofline(w, kernel_ms, n_frames=1, n_dv=1, mixed=False):
    """Achieved rate and roofline fraction of every timed kernel (algorithmic
    work of its own body x n_frames over its average duration)."""
    out = {}
    for name, ms in kernel_ms.items():
        bound, work, unit = kernel_work(w, name, n_frames, n_dv, mixed)
        scale = 1e9 if bound == "hbm" else 1e12
        achieved = work / (ms * 1e-3) / scale
        peak = peak_of(bound, mixed)
        out[name] = dict(us=round(ms * 1e3, 2), bound=bound, achieved=round(achieved, 4), unit=unit,
                         frac=round(achieved / peak, 5), roof_us=round(work / scale / peak * 1e6, 4))
    return out


def step_fraction(w, kernel_ms, ms_step):
    """Whole one-frame step: the sum over the step's kernel bodies of the time
    each would take at its roofline, divided by the measured step time."""
    roof_s = 0.0
    for name in kernel_ms:
        bound, work, _ = kernel_work(w, name)
        roof_s += work / (1e9 if bound == "hbm" else 1e12) / peak_of(bound)
    return dict(roofline_us=roof_s * 1e6, measured_us=ms_step * 1e3, frac=roof_s / (ms_step * 1e-3),
                kernels=sorted(kernel_ms))


# The roofline kernel: the site-site pair forces, the step's largest
# arithmetic workload (k_e Q Q' g0 over every site pair within r_c).  In the
# step its workgroups ride in the field's z-pass launch; it is timed alone
# through the stand-alone kernel with the same body (k_site_pairs), which
# the step never launches, so its rocprofv3 average is its own.
ROOFLINE_KERNEL = "site_pairs"

# HBM traffic of one k_site_pairs launch (doubled paper cell), from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE), each
# scaled by the same counter's reading for a 256 MiB device copy; valid
# only while the kernel's sources are the ones measured (hash below).
TRAFFIC = {"site_pairs": {"bytes": 413666, "sources_sha256": "16b0805e7eb124f4516189d0cdb35401f2f6c7fce4391fbf60ad96bf17cc99ef"}}
TRAFFIC_SOURCES = ["csrc/pairs.h", "csrc/tiles.h", "csrc/k_realspace.hip", "csrc/common.h", "csrc/erfcx_cheb.h"]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2201_12963_amd")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name):
    t = TRAFFIC.get(name)
    if not t or t["bytes"] is None or t["sources_sha256"] != sources_sha256():
        return None
    return t["bytes"]


def roofline(w, kernel_ms, ms_step):
    """Roofline entry for the site-site pair kernel, timed alone, plus the
    whole-step fraction and every kernel's own fraction."""
    name = ROOFLINE_KERNEL
    ms = kernel_ms[name]
    bound, work, unit = kernel_work(w, name)
    scale = 1e9 if bound == "hbm" else 1e12
    achieved = work / (ms * 1e-3) / scale
    peak = peak_of(bound)
    pg0, pg1 = pair_counts(w)
    return dict(kernel=name, bound=bound, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak,
                traffic=measured_traffic(name), avg_us=ms * 1e3, work_per_launch=work,
                work_basis=f"{pg0} unordered site pairs within r_c x {FLOPS_PAIR_G0} FLOP",
                step=step_fraction(w, kernel_ms, ms_step),
                per_kernel=per_kernel_roofline(w, kernel_ms))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_steps(cpm, w, A, S, es, traj, start, n):
    t0 = time.perf_counter()
    for k in range(n):
        cpm.step(w, A, S, es, site_xyz=traj[(start + k) % traj.shape[0]])
    return (time.perf_counter() - t0) / n


def cpu_baseline(w, traj, steps_per_rep=2, reps=5, parity=None):
    """The oracle (FP64 NumPy/SciPy, PPPM) on a bounded sample of the same
    loop: the median of `reps` repeats of `steps_per_rep` consecutive steps
    on all the host's BLAS threads, and the same with one thread.  With
    `parity` (a dict of GPU results of the precision form), the oracle also
    computes that step and the GPU's per-result error against it is returned."""
    from oracle import cpm
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    A, S = cpm.build(w)
    es = cpm.Electrostatics(w, "pppm")
    cpm.step(w, A, S, es, site_xyz=traj[0])          # warm-up
    per_step = [_time_steps(cpm, w, A, S, es, traj, 1 + r * steps_per_rep, steps_per_rep) for r in range(reps)]
    with threadpool_limits(limits=1):
        one = [_time_steps(cpm, w, A, S, es, traj, 1 + r, 1) for r in range(reps)]
    out = dict(value=1.0 / float(np.median(per_step)), unit="steps/s", cores=threads, kind="oracle",
               cpu_model=cpu_model(), os_cpu_count=os.cpu_count(),
               single_core_steps_per_s=1.0 / float(np.median(one)),
               sample=f"median of {reps} repeats of {steps_per_rep} consecutive steps of the same random-walk "
                      f"loop ({w.geometry}, N_e={w.n_elec}, N_l={w.n_site}) on {threads} BLAS threads; "
                      f"single core: median of {reps} single steps; A and S precomputed outside the timing")
    if parity is not None:
        out["precision_form_vs_oracle"] = precision_parity(cpm, parity)
    return out


def precision_parity(cpm, g):
    """Per-result error of the precision form's last GPU step against the oracle."""
    w, x = g["workload"], g["site_xyz"]
    A, S = cpm.build(w)
    ref = cpm.step(w, A, S, cpm.Electrostatics(w, "pppm"), site_xyz=x)
    out = {}
    for label in ("fp64", "mixed"):
        r = g[label]
        out[label] = dict(
            q_max_err_e=float(np.abs(r["q"] - ref["q"]).max()),
            f_rel_rms=float(np.sqrt(np.mean((r["f"] - ref["f"]) ** 2) / np.mean(ref["f"] ** 2))),
            u_coul_err_ev=float(abs(r["e"][0] - ref["u_coul"])),
            e_cp_err_ev=float(abs(r["e"][1] - ref["e_cp"])))
    return out


def precision_form(torch, steps=200, warmup=20):
    """Large cell (N_e = 3520, N_l = 5120): FP64 and mixed steps/s and the mixed errors
    against FP64 on the GPU (the errors against the oracle are taken in the CPU leg)."""
    from workloads import make_workload, random_walk
    w = make_workload("large", "ff")
    traj = random_walk(w, 200)
    r64 = gpu_steps(torch, w, traj, steps, warmup, precision=0)
    r32 = gpu_steps(torch, w, traj, steps, warmup, precision=1)
    dq = float(np.abs(r32["q"] - r64["q"]).max())
    df = float(np.sqrt(np.mean((r32["f"] - r64["f"]) ** 2) / np.mean(r64["f"] ** 2)))
    last = traj[(steps - 1) % traj.shape[0]]
    state = dict(workload=w, site_xyz=last,
                 fp64={k: r64[k] for k in ("q", "f", "e")}, mixed={k: r32[k] for k in ("q", "f", "e")})
    return dict(workload="6.8x6.8x12.625 nm finite field, N_e=3520, N_l=5120, PPPM 36x36x64",
                fp64_steps_per_s=1000.0 * steps / r64["ms_total"],
                mixed_steps_per_s=1000.0 * steps / r32["ms_total"],
                mixed_vs_fp64_q_max_err_e=dq, mixed_vs_fp64_f_rel_rms=df,
                mixed_vs_fp64_u_err_ev=float(abs(r32["e"][0] - r64["e"][0]))), state


def batched_form(torch, n_frames=4096, n_dv=32, reps=3):
    """4096 perturbed frames x 32 dV of the finite-field paper cell per call; (frame, dV) pairs per second."""
    from workloads import make_workload, perturbed_frames
    w = make_workload("paper", "ff")
    frames = torch.tensor(perturbed_frames(w, n_frames), dtype=torch.float64, device="cuda")
    dvs = np.linspace(0.0, 4.0, n_dv)
    out = {}
    for prec, label in ((0, "fp64"), (1, "mixed")):
        ctx, stream = make_ctx(torch, w, prec)
        q = torch.empty((n_frames, n_dv, w.n_elec), dtype=torch.float64, device="cuda")
        f = torch.empty((n_frames, n_dv, 3, w.n_site), dtype=torch.float64, device="cuda")
        e = torch.empty((n_frames, n_dv, 2), dtype=torch.float64, device="cuda")
        with torch.cuda.stream(stream):
            ctx.solve_batch(frames, dvs, q, f, e)
        stream.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            a.record(stream)
            for _ in range(reps):
                ctx.solve_batch(frames, dvs, q, f, e)
            b.record(stream)
        stream.synchronize()
        ms = a.elapsed_time(b) / reps
        from paper_2201_12963_amd.binding import BUF_BATCH_CHUNK
        tuned = ctx.get_buffer(BUF_BATCH_CHUNK)
        out[label] = dict(frames_per_s=n_frames * n_dv / (ms * 1e-3), ms_per_batch=ms,
                          frames_per_launch=int(tuned[0]),
                          launch_shapes={"site_pair_tiles_per_cell": int(tuned[1]),
                                         "xy_planes_per_workgroup": "as many as fit" if tuned[2] == 0 else int(tuned[2])})
        out[label + "_q"] = q[:, 7].cpu().numpy()
        # every kernel of the batch timed alone (the last launch of each, over
        # frames_per_launch frames)
        out[label + "_kernels"] = per_kernel_roofline(w, kernel_times(torch, ctx, stream, 3, warm=1),
                                                      out[label]["frames_per_launch"] or n_frames, n_dv,
                                                      mixed=prec == 1)
        ctx.close()
        del q, f, e
        torch.cuda.empty_cache()
    dq = float(np.abs(out["mixed_q"] - out["fp64_q"]).max())
    return dict(workload=f"{n_frames} frames (sigma=0.05 nm perturbations) x {n_dv} dV in [0, 4] V, "
                         "finite-field paper cell; a unit is one (frame, dV) pair with q, F and U",
                fp64_frames_per_s=out["fp64"]["frames_per_s"], fp64_ms_per_batch=out["fp64"]["ms_per_batch"],
                mixed_frames_per_s=out["mixed"]["frames_per_s"], mixed_ms_per_batch=out["mixed"]["ms_per_batch"],
                mixed_vs_fp64_q_max_err_e=dq,
                frames_per_launch={"fp64": out["fp64"]["frames_per_launch"], "mixed": out["mixed"]["frames_per_launch"]},
                launch_shapes={"fp64": out["fp64"]["launch_shapes"], "mixed": out["mixed"]["launch_shapes"]},
                fp64_per_kernel=out["fp64_kernels"],
                mixed_per_kernel=out["mixed_kernels"])


def geometry_form(torch, ff_steps_per_s, dc_steps_per_s, steps=400, warmup=40):
    """The paper's cost comparison on one GPU: the slab geometry (z period 3x
    the cell, charged-sheet correction, mesh 18 x 18 x 192 at the finite-field
    spacing) against the fully periodic finite field and doubled cell.  The
    doubled cell holds two independent cells, so its steps count twice per
    simulated cell (as the paper counts its nanoseconds)."""
    from workloads import make_workload, random_walk
    w = make_workload("paper", "slab")
    traj = random_walk(w, 200)
    r = gpu_steps(torch, w, traj, steps, warmup)
    slab = 1000.0 * steps / r["ms_total"]
    return dict(workload="paper-shaped cell in slab geometry: 3.4x3.4x37.875 nm period (cell 12.625 nm + "
                         "empty space), N_e=880, N_l=1280, PPPM 18x18x192 order 5, dipole correction",
                slab_steps_per_s=slab, finite_field_steps_per_s=ff_steps_per_s,
                doubled_cell_cell_steps_per_s=2.0 * dc_steps_per_s,
                finite_field_over_slab=ff_steps_per_s / slab, doubled_cell_over_slab=2.0 * dc_steps_per_s / slab)


def three_layer_form(torch, n_frames=4096, n_dv=32, reps=3):
    """Re-solving snapshots with all three graphene sheets charged (N_e = 2640,
    finite field), batched: (frame, dV) pairs per second, and the share of
    each electrode's net charge on its nearest sheet at the largest dV."""
    from workloads import make_workload, perturbed_frames
    w = make_workload("paper", "ff", layers=3)
    frames = torch.tensor(perturbed_frames(w, n_frames), dtype=torch.float64, device="cuda")
    dvs = np.linspace(0.0, 4.0, n_dv)
    ctx, stream = make_ctx(torch, w)
    q = torch.empty((n_frames, n_dv, w.n_elec), dtype=torch.float64, device="cuda")
    f = torch.empty((n_frames, n_dv, 3, w.n_site), dtype=torch.float64, device="cuda")
    e = torch.empty((n_frames, n_dv, 2), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        ctx.solve_batch(frames, dvs, q, f, e)
    stream.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        for _ in range(reps):
            ctx.solve_batch(frames, dvs, q, f, e)
        b.record(stream)
    stream.synchronize()
    ms = a.elapsed_time(b) / reps
    qh = q[:, -1].cpu().numpy()
    share = []
    for side in (-1, 1):
        m = w.elec_side == side
        share.append(qh[:, m & (w.elec_layer == 0)].sum(-1) / qh[:, m].sum(-1))
    share = np.concatenate(share)
    from paper_2201_12963_amd.binding import BUF_BATCH_CHUNK
    chunk = int(ctx.get_buffer(BUF_BATCH_CHUNK)[0]) or n_frames
    kern = per_kernel_roofline(w, kernel_times(torch, ctx, stream, 3, warm=1), chunk, n_dv)
    ctx.close()
    del q, f, e
    torch.cuda.empty_cache()
    return dict(workload=f"{n_frames} frames x {n_dv} dV of the finite-field paper cell with all three sheets of "
                         "each electrode charged (N_e=2640, N_l=1280)",
                fp64_frames_per_s=n_frames * n_dv / (ms * 1e-3), fp64_ms_per_batch=ms, frames_per_launch=chunk,
                nearest_sheet_share_at_4V={"min": float(share.min()), "mean": float(share.mean())},
                fp64_per_kernel=kern)


def md_form(torch, steps=500, warmup=50):
    """The constant-potential MD loop (velocity Verlet 2 fs, Nose-Hoover 400 K,
    rigid cations, Lennard-Jones, charges every fifth step) on the paper cell
    in finite-field, doubled-cell and slab geometry: MD steps/s and simulated
    ns per day; the doubled cell counts twice (two independent cells, as the
    paper counts its cost)."""
    from paper_2201_12963_amd import MDLoop
    from workloads import make_workload, md_setup
    out = {}
    for geo in ("ff", "dc", "slab"):
        w = make_workload("paper", geo)
        setup = md_setup(w)
        ctx, stream = make_ctx(torch, w)
        mdl = MDLoop(ctx, setup)
        rng = np.random.default_rng(17)
        v0 = rng.normal(0.0, 1.0, (3, w.n_site)) * np.sqrt(0.0083144626 * setup.temperature / setup.site_mass)
        x = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
        v = torch.tensor(v0, dtype=torch.float64, device="cuda")
        q = torch.empty(w.n_elec, dtype=torch.float64, device="cuda")
        with torch.cuda.stream(stream):
            mdl.run(x, v, w.dv, warmup, q_out=q, thermo=False)
        stream.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            a.record(stream)
            mdl.run(x, v, w.dv, steps, q_out=q, thermo=False)
            b.record(stream)
        stream.synchronize()
        if ctx.sync_status() != 0:
            raise RuntimeError("kernel status flag raised during the MD loop")
        ms = a.elapsed_time(b) / steps
        per_cell = 2.0 if geo == "dc" else 1.0
        out[geo] = dict(steps_per_s=1000.0 / ms, us_per_step=ms * 1e3,
                        ns_per_day=per_cell * 1000.0 / ms * setup.dt * 1e-3 * 86400.0)
        mdl.close()
        ctx.close()
    return dict(workload="paper-shaped cell, 320 ion pairs (640 in the doubled cell), rigid 3-site cations, "
                         "Lennard-Jones with all three graphene sheets (synthetic parameters), 2 fs steps, "
                         "charges every 5 steps", **out)


def gradient_form(torch, reps=50):
    from workloads import make_workload
    w = make_workload("large", "ff")
    ctx, stream = make_ctx(torch, w)
    x = torch.tensor(w.site_xyz, dtype=torch.float64, device="cuda")
    t = torch.tensor(np.random.default_rng(5).normal(0, 0.01, w.n_elec), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        ctx.grad(x, w.dv, t)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ctx.grad(x, w.dv, t)
        b.record(stream)
    stream.synchronize()
    ms = a.elapsed_time(b) / reps
    ctx.close()
    return dict(workload="large finite-field cell, d(loss)/d(5120 x 3 positions, dV)",
                evals_per_s=1000.0 / ms, ms_per_eval=ms)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--only", choices=("precision", "batched", "gradient", "three_layer", "md"),
                    help="run only this form and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this path runs on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import make_workload, random_walk

    if args.only:
        form = {"precision": lambda t: precision_form(t)[0], "batched": batched_form,
                "gradient": gradient_form, "three_layer": three_layer_form, "md": md_form}[args.only]
        print(json.dumps({args.only: form(torch)}), flush=True)
        return

    n_traj = min(max(args.steps, 1), 1000)
    wd = make_workload("paper", "dc")
    trajd = random_walk(wd, n_traj)
    rd = gpu_steps(torch, wd, trajd, args.steps, args.warmup, profile_kernels=True)
    wf = make_workload("paper", "ff")
    trajf = random_walk(wf, n_traj)
    rf = gpu_steps(torch, wf, trajf, args.steps, args.warmup)

    ms_step = rd["ms_total"] / args.steps
    line = {
        "metric": "CPM charge-solve+force steps/s; batched frames/s at <=1e-6 e charge error",
        "value": 1000.0 / ms_step,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "paper-shaped cell, doubled cell: 3.4x3.4x25.25 nm, N_e=1760 charged electrode "
                        "atoms, N_l=2560 sites (640 ion pairs), PPPM 18x18x128 order 5, alpha=2.21/nm, "
                        "rcut=1.2 nm, dV=2 V, random-walk loop sigma=0.005 nm/step",
            "finite_field_steps_per_s": 1000.0 * args.steps / rf["ms_total"],
            "finite_field_workload": "same cell, finite field: 3.4x3.4x12.625 nm, N_e=880, N_l=1280, "
                                     "PPPM 18x18x64",
        },
        "roofline": roofline(wd, rd["kernel_ms"], ms_step),
    }
    precision_state = None
    if not args.no_forms:
        prec, precision_state = precision_form(torch)
        line["forms"] = {
            "precision": prec,
            "batched": batched_form(torch),
            "gradient": gradient_form(torch),
            "geometries": geometry_form(torch, line["config"]["finite_field_steps_per_s"], line["value"]),
            "three_layer": three_layer_form(torch),
            "md": md_form(torch),
        }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wd, trajd, parity=precision_state)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
