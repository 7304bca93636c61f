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
REPLAYS = int(os.environ.get("CPM_BENCH_REPLAYS", "200"))

# Algorithmic FP64 operation counts of the per-pair formulas (erfc ~ 20 and
# exp ~ 10 operations as polynomial/rational evaluations, plus the arithmetic
# around them): potential g1 pair 50, force g0 pair 50, force g1 pair 80.
FLOPS_PAIR_B, FLOPS_PAIR_G0, FLOPS_PAIR_G1 = 50, 50, 80


def count_pairs(a, b, box, rcut, same=False):
    """Number of (a, b) pairs within rcut (minimum image; the cells used here are >= 2 rcut)."""
    n = 0
    for i0 in range(0, a.shape[1], 512):
        d = a[:, i0:i0 + 512, None] - b[:, None, :]
        d -= box[:, None, None] * np.round(d / box[:, None, None])
        r2 = np.einsum("kab,kab->ab", d, d)
        n += int(np.count_nonzero(r2 < rcut * rcut))
    if same:
        n -= a.shape[1]
    return n


def kernel_work(w, name, n_frames=1):
    """(bound, algorithmic work of one launch over n_frames frames, unit) of a
    step kernel.  Bytes count frame-independent tables (S, S c, electrode
    stencils, the influence function) once per launch and per-frame data
    once per frame; FLOP counts are per frame."""
    P3 = w.order ** 3
    M = int(np.prod(w.mesh))
    ne, nl = w.n_elec, w.n_site
    if name == "site_pairs":
        pg0 = count_pairs(w.site_xyz, w.site_xyz, w.box, w.rcut, same=True)
        return "alu", n_frames * pg0 * FLOPS_PAIR_G0, "TFLOP/s"
    if name == "site_forces":
        pg1 = count_pairs(w.site_xyz, w.elec_xyz, w.box, w.rcut)
        return "alu", n_frames * (pg1 * FLOPS_PAIR_G1 + nl * P3 * 6), "TFLOP/s"
    if name == "real_b":
        return "alu", n_frames * count_pairs(w.elec_xyz, w.site_xyz, w.box, w.rcut) * FLOPS_PAIR_B, "TFLOP/s"
    if name == "charges":           # S streamed once; b read, Q0 and q written per frame
        return "hbm", 8 * ne * ne + n_frames * 8 * 3 * ne, "GB/s"
    if name.startswith("fft_z"):    # complex mesh read and written (+ G once)
        return "hbm", M * 8 + n_frames * M * 16 * 2, "GB/s"
    if name.startswith("fft_xy"):   # real plane in, complex plane out (or back)
        return "hbm", n_frames * M * (8 + 16), "GB/s"
    if name == "spread_elec":       # stencil table once; q read, mesh written per frame
        return "hbm", ne * P3 * 12 + n_frames * (ne * 8 + M * 8), "GB/s"
    if name == "gather_b":          # stencil table once; mesh read, b written per frame
        return "hbm", ne * P3 * 12 + n_frames * (M * 8 + ne * 16), "GB/s"
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


def per_kernel_roofline(w, kernel_ms, n_frames=1):
    """Achieved rate and roofline fraction of every timed kernel (algorithmic
    work of its own body x n_frames over its average duration)."""
    out = {}
    for name, ms in kernel_ms.items():
        bound, work, unit = kernel_work(w, name, n_frames)
        if bound == "hbm":
            achieved, peak = work / (ms * 1e-3) / 1e9, HBM_PEAK_GBS
        else:
            achieved, peak = work / (ms * 1e-3) / 1e12, FP64_PEAK_TFLOPS
        out[name] = dict(us=round(ms * 1e3, 2), bound=bound, achieved=round(achieved, 4), unit=unit,
                         frac=round(achieved / peak, 5))
    return out


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
TRAFFIC = {"site_pairs": {"bytes": 444672, "sources_sha256": "ec136434e70f5d904e41b49d233d30faa9aa639183e5d39585246f019f949cb6"}}
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


def roofline(w, kernel_ms):
    """Roofline entry for the site-site pair kernel, timed alone."""
    name = ROOFLINE_KERNEL
    ms = kernel_ms[name]
    bound, work, unit = kernel_work(w, name)
    if bound == "hbm":
        achieved = work / (ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
    else:
        achieved = work / (ms * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS
    return dict(kernel=name, bound=bound, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak,
                traffic=measured_traffic(name), avg_us=ms * 1e3, work_per_launch=work,
                per_kernel=per_kernel_roofline(w, kernel_ms))


def cpu_baseline(w, traj, budget_s=20.0):
    """The oracle (FP64 NumPy/SciPy, PPPM) on a bounded sample of the same loop."""
    from oracle import cpm
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    A, S = cpm.build(w)
    es = cpm.Electrostatics(w, "pppm")
    cpm.step(w, A, S, es, site_xyz=traj[0])          # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        cpm.step(w, A, S, es, site_xyz=traj[(n + 1) % traj.shape[0]])
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 50:
            break
    return dict(value=n / el, unit="steps/s", cores=threads, kind="oracle",
                sample=f"{n} consecutive steps of the same random-walk loop ({w.geometry}, "
                       f"N_e={w.n_elec}, N_l={w.n_site}), A and S precomputed outside the timing")


def precision_form(torch, steps=200, warmup=20):
    """Large cell (N_e = 3520, N_l = 5120): FP64 and mixed steps/s and the mixed errors."""
    from workloads import make_workload, random_walk
    w = make_workload("large", "ff")
    traj = random_walk(w, 200)
    r64 = gpu_steps(torch, w, traj, steps, warmup, precision=0)
    r32 = gpu_steps(torch, w, traj, steps, warmup, precision=1)
    dq = float(np.abs(r32["q"] - r64["q"]).max())
    df = float(np.sqrt(np.mean((r32["f"] - r64["f"]) ** 2) / np.mean(r64["f"] ** 2)))
    return dict(workload="6.8x6.8x12.625 nm finite field, N_e=3520, N_l=5120, PPPM 36x36x64",
                fp64_steps_per_s=1000.0 * steps / r64["ms_total"],
                mixed_steps_per_s=1000.0 * steps / r32["ms_total"],
                mixed_vs_fp64_q_max_err_e=dq, mixed_vs_fp64_f_rel_rms=df,
                mixed_vs_fp64_u_err_ev=float(abs(r32["e"][0] - r64["e"][0])))


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
        out[label] = dict(frames_per_s=n_frames * n_dv / (ms * 1e-3), ms_per_batch=ms,
                          frames_per_launch=int(ctx.get_buffer(BUF_BATCH_CHUNK)[0]))
        out[label + "_q"] = q[:, 7].cpu().numpy()
        # every kernel of the batch timed alone (the last launch of each, over
        # frames_per_launch frames)
        out[label + "_kernels"] = per_kernel_roofline(w, kernel_times(torch, ctx, stream, 3, warm=1),
                                                      out[label]["frames_per_launch"] or n_frames)
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
                fp64_per_kernel=out["fp64_kernels"],
                mixed_per_kernel=out["mixed_kernels"])


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
    ap.add_argument("--only", choices=("precision", "batched", "gradient"),
                    help="run only this form and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this path runs on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import make_workload, random_walk

    if args.only:
        form = {"precision": precision_form, "batched": batched_form, "gradient": gradient_form}[args.only]
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
        "roofline": roofline(wd, rd["kernel_ms"]),
    }
    if not args.no_forms:
        line["forms"] = {
            "precision": precision_form(torch),
            "batched": batched_form(torch),
            "gradient": gradient_form(torch),
        }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wd, trajd)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
