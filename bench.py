"""Throughput of the batched Gerchberg extension + Fourier reconstruction on one MI355X.

Workload: 4096 independent 40x40 Shack-Hartmann frames (SPHERE-like geometry,
von Karman screens D = 8 m, r0 = 0.15 m, L0 = 25 m, slope noise 0.05 rad),
padded to 80x80, 10 Gerchberg iterations, Eq. 5 after the loop, MMSE final
filter; float32 slopes in, float32 phase out, one launch per step.  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1705_04298_amd import inputs as I  # noqa: E402

N_SUB, N_GRID, N_ITER, BATCH = 40, 80, 10, 4096
FP32_VECTOR_PEAK = 157.3e12  # MI355X published FP32 vector peak [flop/s]


def algorithmic_flops_per_frame(N: int, n_iter: int) -> float:
    """Per-frame work of the paper's formulation (Eq. 8 made concrete): two complex
    N^2-point FFTs per iteration and for the final step at 5 M log2 M flops each,
    ~24 flop per frequency for the in-loop filter and gradient, ~16 for the final one."""
    M = N * N
    fft = 5.0 * M * math.log2(M)
    return n_iter * (2 * fft + 24 * M) + (2 * fft + 16 * M)


def _gen(args):
    start, count = args
    return I.make_batch(I.SPHERE_40_BATCH, count, start=start, dtype=np.float32)


def make_inputs(B: int, workers: int) -> np.ndarray:
    chunk = 64
    jobs = [(s, min(chunk, B - s)) for s in range(0, B, chunk)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_gen, jobs)
    return np.concatenate(parts, axis=0)


_CPU_SLOPES = None
KERNEL_SOURCES = ("gerchberg_onchip.hip", "fft_lane.h", "onchip.h")
PROFILE = os.path.join(ROOT, "profiles", "gerchberg_onchip_80x80_b4096.md")


def _oracle_frames(idx):
    from oracle import fwr_oracle as O
    p = O.Params(n_sub=N_SUB, n_grid=N_GRID, n_iter=N_ITER, periodic=True, gamma=1.0,
                 noise_var=0.05 ** 2, r0=0.15, L0=25.0, d=0.2)
    mask = I.pupil_mask(N_SUB)
    return [(i, O.reconstruct(_CPU_SLOPES[i].astype(np.float64), mask, p)) for i in idx]


def cpu_baseline(slopes: np.ndarray, workers: int, sample: int):
    """The FP64 oracle, unchanged, over `sample` frames split across `workers` processes.
    Returns the timing record and the oracle's phases (for the parity figure)."""
    global _CPU_SLOPES
    _CPU_SLOPES = slopes
    idx = np.arange(sample)
    parts = [idx[w::workers] for w in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_frames, parts)
        dt = time.perf_counter() - t0
    ref = {i: ph for part in res for i, ph in part}
    rec = {"value": len(ref) / dt, "unit": "frames/s", "cores": workers, "kind": "oracle",
           "sample": f"first {sample} frames of the benchmark batch, FP64 NumPy oracle, "
                     f"{workers} single-threaded worker processes, {dt:.1f} s wall",
           "cpu_model": cpu_model()}
    return rec, ref


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_fingerprint() -> str:
    """Hash of the kernel sources without comments and blank lines (a comment edit does not
    change the kernel the profile measured)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1705_04298_amd", "csrc", name)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def profiled_value(key: str):
    """A per-launch figure (`traffic_bytes_per_launch`, `executed_flop_per_launch`) from the
    committed rocprofv3 summary, if it was taken on these sources."""
    try:
        with open(PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    fields = dict(l.split(":", 1) for l in text.splitlines() if l.startswith(("source_fingerprint:", key + ":")))
    if fields.get("source_fingerprint", "").strip() != kernel_fingerprint():
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def profiled_traffic():
    """HBM bytes per launch from the committed rocprofv3 summary, if it was taken on these sources."""
    return profiled_value("traffic_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cnn", action="store_true", help="uneven workload: plain start for the 40x40 frames")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default launch shape")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes for input generation (0 = up to 16; use 1 under a profiler)")
    ap.add_argument("--workload", choices=("sphere40", "elt128", "uneven", "sinc40", "single", "learned40"),
                    default="sphere40",
                    help="sphere40: the headline 4096 x 40x40 batch; elt128: 128 x 128x128 frames on "
                         "the 256x256 multi-pass path; uneven: the mixed-size closed loop captured in a "
                         "HIP graph; sinc40: the headline batch with the lenslet-averaging slope model; "
                         "single: one grid size alone (--n-sub, --frames, --iters, --model); learned40: "
                         "the learned start on the headline batch (each prints its own line)")
    ap.add_argument("--n-sub", type=int, default=24, help="single workload: lenslets per side (grid 2n)")
    ap.add_argument("--frames", type=int, default=2048, help="single workload: frames per launch")
    ap.add_argument("--iters", type=int, default=N_ITER, help="single / learned40 workload: loop iterations")
    ap.add_argument("--model", choices=("fried", "sinc"), default="fried", help="single workload: slope model")
    ap.add_argument("--graph-steps", type=int, default=1000,
                    help="uneven workload: timed graph replays (one loop step each)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration * (1 << 18), device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
        return
    if args.workload == "elt128":
        return elt_main(args)
    if args.workload == "uneven":
        return uneven_main(args)
    if args.workload == "sinc40":
        return sinc_main(args)
    if args.workload == "single":
        return single_main(args)
    if args.workload == "learned40":
        return learned_main(args)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (frames are independent; see the design notes "
              f"for how the batch shards): --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    if args.gen_workers == 1:
        slopes = I.make_batch(I.SPHERE_40_BATCH, args.batch, dtype=np.float32)
    else:
        slopes = make_inputs(args.batch, args.gen_workers or workers)
    print(f"[bench] generated {args.batch} frames in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    cpu, ref = None, None
    if not args.no_cpu_baseline:
        cpu, ref = cpu_baseline(slopes, workers, min(args.cpu_sample, args.batch))
        print(f"[bench] cpu baseline {cpu['value']:.0f} frames/s", file=sys.stderr, flush=True)

    import torch
    from paper_1705_04298_amd import fwr

    torch.cuda.set_device(0)
    mask = I.pupil_mask(N_SUB)
    plan = fwr.Plan(N_SUB, N_GRID, mask, n_iter=N_ITER, periodic=True, gamma=1.0,
                    noise_var=0.05 ** 2, r0=0.15, L0=25.0, d=0.2, max_batch=args.batch)
    x = torch.from_numpy(slopes).cuda()
    if not args.no_autotune:
        plan.autotune(args.batch)  # launch shape (frames per workgroup) by timing
    threads, fpg, lds = plan.launch_info()
    sched = plan.schedule
    out = torch.empty((args.batch, N_SUB + 1, N_SUB + 1), device="cuda", dtype=torch.float32)
    for _ in range(args.warmup):
        plan.reconstruct(x, out)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_begin.record()
    for k in range(args.steps):
        starts[k].record()
        plan.reconstruct(x, out)
        ends[k].record()
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_begin.elapsed_time(t_end)
    per_launch_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    ms_per_step = total_ms / args.steps
    frames_per_s = args.batch * args.steps / (total_ms / 1e3)

    flops = algorithmic_flops_per_frame(N_GRID, N_ITER) * args.batch
    achieved = flops / (per_launch_ms / 1e3)
    parity = None
    if ref is not None:
        got = out.cpu().numpy().astype(np.float64)
        errs = [np.sqrt(np.mean((got[i] - want) ** 2) / np.mean(want ** 2)) for i, want in ref.items()]
        parity = {"frames": len(errs), "max_rel_rms": float(np.max(errs)),
                  "median_rel_rms": float(np.median(errs)), "tolerance": 1e-5}
    executed = profiled_value("executed_flop_per_launch")
    line = {
        "metric": "frames/s (40x40 SH, 10 Gerchberg iters) + rms phase err vs FP64 oracle",
        "value": frames_per_s,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4096 frames 40x40 SH (Fried), pupil 14% obstruction, padded 80x80, "
                               "10 Gerchberg iterations + Eq.5 + MMSE, von Karman D=8m r0=0.15m L0=25m, "
                               "noise 0.05 rad",
                   "batch": args.batch, "n_sub": N_SUB, "n_grid": N_GRID, "n_iter": N_ITER,
                   "threads_per_group": threads, "frames_per_group": fpg, "lds_bytes_per_group": lds,
                   "fft_radix_schedule": sched},
        "rms_phase_error_vs_oracle": parity,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK, "traffic": profiled_traffic(),
                     "kernel_ms": per_launch_ms,
                     "flops_per_frame": algorithmic_flops_per_frame(N_GRID, N_ITER),
                     # FP32 work the kernel actually executes (SQ_INSTS_VALU_{FMA,ADD,MUL}_F32 from the
                     # committed profile): the pruned, frame-paired loop does far less than the
                     # algorithmic count above
                     "executed_tflops": (None if executed is None else executed / (per_launch_ms / 1e3) / 1e12)},
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(line), flush=True)


def elt_main(args):
    """128 frames of 128x128 subapertures (D = 39 m) padded to 256x256, 20 iterations, multi-pass.
    HBM-bound: roofline against 8 TB/s with 2 MiB per frame-iteration + 128 KiB of slopes."""
    import torch
    from paper_1705_04298_amd import fwr
    B, n, N, n_iter = 128, 128, 256, 20
    slopes = I.make_batch(I.ELT_128, B, dtype=np.float32)
    torch.cuda.set_device(0)
    plan = fwr.Plan(n, N, I.pupil_mask(n), n_iter=n_iter, periodic=True, gamma=1.0,
                    noise_var=0.05 ** 2, r0=0.15, L0=25.0, d=39.0 / n, max_batch=B)
    if not args.no_autotune:
        plan.autotune(B)  # the loop's launch shape: per pass (16 or 64 threads per line) or persistent
    x = torch.from_numpy(slopes).cuda()
    out = torch.empty((B, n + 1, n + 1), device="cuda", dtype=torch.float32)
    for _ in range(args.warmup):
        plan.reconstruct(x, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.reconstruct(x, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    alg_bytes = B * (n_iter * 2 * 2 ** 20 + 2 * 2 ** 16)
    tpl = 64 if plan.schedule == 1 else 16
    loop_shape = "one persistent launch" if plan.schedule == 2 else "one launch per pass"
    plan.close()
    print(json.dumps({"metric": "frames/s (128x128 SH, 256x256 grid, 20 Gerchberg iters)",
                      "value": B / (ms / 1e3), "unit": "frames/s", "ms_per_step": ms, "steps": args.steps,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"{B} frames 128x128 -> 256x256, 20 iterations + Eq.5 + MMSE",
                                 "column_pass_threads_per_line": tpl, "loop": loop_shape},
                      "roofline": {"bound": "hbm", "achieved": alg_bytes / (ms / 1e3) / 1e9, "peak": 8000.0,
                                   "unit": "GB/s", "frac": alg_bytes / (ms / 1e3) / 8e12, "traffic": None}}),
          flush=True)


def _gen_sinc(args):
    start, count = args
    return I.make_batch(I.SPHERE_40_SINC, count, start=start, dtype=np.float32)


def _oracle_sinc(idx):
    from oracle import fwr_oracle as O
    p = O.Params(n_sub=N_SUB, n_grid=N_GRID, n_iter=N_ITER, periodic=True, model="sinc")
    mask = I.pupil_mask(N_SUB)
    return [(i, O.reconstruct(_CPU_SLOPES[i].astype(np.float64), mask, p)) for i in idx]


def sinc_main(args):
    """The headline batch (4096 x 40x40 -> 80x80, 10 iterations + Eq. 5 + MMSE) with the
    lenslet-averaging slope model of Eq. 4 on the Fourier-domain kernel; parity against the FP64
    oracle over a sample of the batch."""
    global _CPU_SLOPES
    import torch
    from paper_1705_04298_amd import fwr
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    if args.gen_workers:
        workers = args.gen_workers
    jobs = [(s0, min(64, args.batch - s0)) for s0 in range(0, args.batch, 64)]
    sample = min(args.cpu_sample, args.batch)
    if workers == 1:  # no worker processes (under a profiler)
        slopes = np.concatenate([_gen_sinc(j) for j in jobs], axis=0)
        _CPU_SLOPES = slopes
        ref = dict(_oracle_sinc(np.arange(sample)))
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            slopes = np.concatenate(pool.map(_gen_sinc, jobs), axis=0)
        _CPU_SLOPES = slopes
        parts = [np.arange(sample)[w::workers] for w in range(workers)]
        with mp.get_context("fork").Pool(workers) as pool:
            ref = {i: ph for part in pool.map(_oracle_sinc, parts) for i, ph in part}
    torch.cuda.set_device(0)
    plan = fwr.Plan(N_SUB, N_GRID, I.pupil_mask(N_SUB), n_iter=N_ITER, periodic=True, max_batch=args.batch,
                    model="sinc")
    x = torch.from_numpy(slopes).cuda()
    if not args.no_autotune:
        plan.autotune(args.batch)
    threads, fpg, lds = plan.launch_info()
    sched = plan.schedule
    out = torch.empty((args.batch, N_SUB + 1, N_SUB + 1), device="cuda")
    for _ in range(args.warmup):
        plan.reconstruct(x, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.reconstruct(x, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    got = out.cpu().numpy().astype(np.float64)
    errs = [np.sqrt(np.mean((got[i] - w) ** 2) / np.mean(w ** 2)) for i, w in ref.items()]
    flops = algorithmic_flops_per_frame(N_GRID, N_ITER) * args.batch
    plan.close()
    print(json.dumps({
        "metric": "frames/s (40x40 SH, 10 Gerchberg iters, lenslet-averaging slope model)",
        "value": args.batch / (ms / 1e3), "unit": "frames/s", "ms_per_step": ms, "steps": args.steps,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "4096 frames 40x40 SH, lenslet-averaging (sinc) slopes of von Karman screens, "
                               "padded 80x80, 10 iterations + Eq.5 + MMSE", "model": "sinc",
                   "threads_per_group": threads, "frames_per_group": fpg, "lds_bytes_per_group": lds,
                   "fft_radix_schedule": sched},
        "rms_phase_error_vs_oracle": {"frames": len(errs), "max_rel_rms": float(np.max(errs)),
                                      "median_rel_rms": float(np.median(errs)), "tolerance": 1e-5},
        "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / FP32_VECTOR_PEAK, "traffic": None},
    }), flush=True)


def _timed(fn, steps, warmup):
    """Mean ms per call of `fn` between HIP events on the current stream, after `warmup` calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def single_main(args):
    """One grid size alone: `--frames` frames of `--n-sub` x `--n-sub` lenslets padded to 2n,
    `--iters` iterations + Eq. 5 + MMSE, slopes resident in HBM.  Fried frames come from the device
    generator (D = 8 m, or 39 m for n = 128), lenslet-averaging frames from the host generator.
    On-chip grids: FP32 roofline of the algorithmic FFT work; the 256 x 256 grid: HBM roofline of
    2 MiB per frame and iteration (two round trips of a 512 KiB complex field)."""
    import dataclasses
    import torch
    from paper_1705_04298_amd import fwr
    n, B, it = args.n_sub, args.frames, args.iters
    N = 2 * n
    D = 39.0 if n == 128 else 8.0
    torch.cuda.set_device(0)
    plan = fwr.Plan(n, N, I.pupil_mask(n), n_iter=it, periodic=True, gamma=1.0, noise_var=0.05 ** 2,
                    r0=0.15, L0=25.0, d=D / n, max_batch=B, model=args.model)
    if args.model == "fried":
        x, _ = plan.generate(B, 0x5EED_0517, r0=0.15, L0=25.0, sigma=0.05)
    else:
        w = dataclasses.replace(I.SPHERE_40_SINC, n_sub=n, diameter=D, screen_size=512 if N > 128 else 256,
                                config_id=8)
        x = torch.from_numpy(I.make_batch(w, B, dtype=np.float32)).cuda()
    if not args.no_autotune:
        plan.autotune(B)
    threads, fpg, lds = plan.launch_info()
    sched = plan.schedule
    out = torch.empty((B, n + 1, n + 1), device="cuda")
    ms = _timed(lambda: plan.reconstruct(x, out), args.steps, args.warmup)
    if N <= 128:
        flops = algorithmic_flops_per_frame(N, it) * B
        roof = {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / FP32_VECTOR_PEAK, "traffic": None}
    else:
        alg = B * (it * 2 * 2 ** 20 + 2 * n * n * 4 + (n + 1) ** 2 * 4)
        roof = {"bound": "hbm", "achieved": alg / (ms / 1e3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                "frac": alg / (ms / 1e3) / 8e12, "traffic": None}
    plan.close()
    print(json.dumps({"metric": f"frames/s ({n}x{n} SH, {N}x{N} grid, {it} Gerchberg iters, {args.model} model)",
                      "value": B / (ms / 1e3), "unit": "frames/s", "ms_per_step": ms, "steps": args.steps,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"{B} frames {n}x{n} -> {N}x{N}, {it} iterations + Eq.5 + MMSE",
                                 "threads_per_group": threads, "frames_per_group": fpg,
                                 "lds_bytes_per_group": lds, "fft_radix_schedule": sched},
                      "roofline": roof}), flush=True)


def cnn_forward_bytes_per_frame(N: int) -> int:
    """Algorithmic HBM bytes of one network forward per N x N frame: the slopes in, the features
    (8 BF16 channels), each layer's BF16 input and output activations read / written once (32
    channels; the last layer writes 2 FP32 channels)."""
    px = N * N
    feats = 2 * N_SUB * N_SUB * 4 + px * 8 * 2
    layers = px * (8 * 2 + 32 * 2) + 5 * px * (32 * 2 + 32 * 2) + px * (32 * 2 + 2 * 4)
    return feats + layers


def learned_main(args):
    """The learned start on the headline batch (4096 x 40x40 -> 80x80): the network forward alone
    (roofline: HBM, each activation read and written once per layer), the network + `--iters`
    iterations, the plain 10-iteration loop, and the one-call learned reconstruction with the plain
    loop as fallback (threshold twice the plain-10 median residual)."""
    import torch
    from paper_1705_04298_amd import fwr
    from paper_1705_04298_amd import learned as L
    B = args.batch
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    if args.gen_workers == 1:  # no worker processes (under a profiler)
        slopes = I.make_batch(I.SPHERE_40_BATCH, B, dtype=np.float32)
    else:
        slopes = make_inputs(B, args.gen_workers or workers)
    torch.cuda.set_device(0)
    mask = I.pupil_mask(N_SUB)
    x = torch.from_numpy(slopes).cuda()
    params = np.load(os.path.join(ROOT, "paper_1705_04298_amd", "weights", "cnn_40x40_fried.npz"))["params"]
    net = fwr.CNN(N_SUB, N_GRID, mask, max_batch=B, input_scale=L.INPUT_SCALE)
    net.set_params(params)
    start = torch.empty((B, 2, N_GRID, N_GRID), device="cuda")
    kw = dict(periodic=True, gamma=1.0, noise_var=0.05 ** 2, r0=0.15, L0=25.0, d=0.2, max_batch=B)
    plan_k = fwr.Plan(N_SUB, N_GRID, mask, n_iter=args.iters, **kw)
    plain = fwr.Plan(N_SUB, N_GRID, mask, n_iter=N_ITER, **kw)
    out = torch.empty((B, N_SUB + 1, N_SUB + 1), device="cuda")
    resid = torch.empty(B, device="cuda")
    ms_net = _timed(lambda: net.forward(x, start), args.steps, args.warmup)
    ms_k = _timed(lambda: (net.forward(x, start), plan_k.reconstruct(x, out, start=start, resid=resid)),
                  args.steps, args.warmup)
    r_k = float(torch.median(resid))
    ms_plain = _timed(lambda: plain.reconstruct(x, out, resid=resid), args.steps, args.warmup)
    r_plain = float(torch.median(resid))
    thr = 2.0 * r_plain
    count = torch.zeros(1, dtype=torch.int32, device="cuda")

    def one_call():
        st = fwr.fwr_reconstruct_learned_noalloc(plan_k.handle, plain.handle, net._h, x.data_ptr(), start.data_ptr(),
                                                 out.data_ptr(), resid.data_ptr(), thr, B, count.data_ptr())
        if st != fwr.FWR_OK:
            raise fwr.FwrError(st, "fwr_reconstruct_learned_noalloc")
    ms_call = _timed(one_call, args.steps, args.warmup)
    nfall = int(count.item())
    flop = B * 2.0 * N_GRID * N_GRID * sum(9 * ci * co for ci, co in L.LAYERS)
    nbytes = B * cnn_forward_bytes_per_frame(N_GRID)
    for h in (net, plan_k, plain):
        h.close()
    print(json.dumps({
        "metric": f"frames/s, learned start + {args.iters} Gerchberg iters (40x40 SH, 80x80 grid)",
        "value": B / (ms_k / 1e3), "unit": "frames/s", "ms_per_step": ms_k, "steps": args.steps,
        "dtype": "bf16 network (FP32 accumulate) + f32 loop", "data": "synthetic",
        "config": {"workload": f"{B} frames 40x40 -> 80x80, CNN start + {args.iters} iterations + Eq.5 + MMSE",
                   "iters": args.iters},
        "median_residual": {"cnn_plus_k": r_k, "plain_10": r_plain},
        "ms": {"network": ms_net, "network_plus_k": ms_k, "plain_10": ms_plain,
               "one_call_with_fallback": ms_call},
        "fallback": {"threshold": thr, "frames_recomputed": nfall, "frames": B},
        "network_mfma_tflops": flop / (ms_net / 1e3) / 1e12,
        "roofline": {"bound": "hbm", "achieved": nbytes / (ms_net / 1e3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": nbytes / (ms_net / 1e3) / 8e12, "traffic": None,
                     "bytes_per_frame": cnn_forward_bytes_per_frame(N_GRID)},
    }), flush=True)


UNEVEN = ((24, 2048, 8.0 / 24), (40, 2048, 8.0 / 40), (64, 512, 8.0 / 64), (128, 64, 39.0 / 128))


def uneven_main(args):
    """Mixed closed loop: 2048 x 24x24, 2048 x 40x40 (learned start), 512 x 64x64, 64 x 128x128 frames,
    each padded 2x, 10 iterations + Eq. 5 + MMSE.  One loop step = fresh frames from the device
    generator (the next frames of each seeded sequence) + the network's start for the 40x40 frames +
    one grouped reconstruction; the step is captured once in a HIP graph and replayed.  Reports
    frames/s over the replays and the per-step latency percentiles (HIP events around each replay)."""
    import torch
    from paper_1705_04298_amd import fwr
    from paper_1705_04298_amd import learned as L
    torch.cuda.set_device(0)
    seed = 0x5EED_0517_0504_298
    plans, xs, outs, ctrs, starts = [], [], [], [], []
    net = None
    for n, B, d in UNEVEN:
        plan = fwr.Plan(n, 2 * n, I.pupil_mask(n), n_iter=N_ITER, periodic=True, gamma=1.0,
                        noise_var=0.05 ** 2, r0=0.15, L0=25.0, d=d, max_batch=B)
        if not args.no_autotune:
            plan.autotune(B)  # frames per workgroup and radix schedule, by timing
        plans.append(plan)
        xs.append(torch.empty((B, 2, n, n), device="cuda"))
        outs.append(torch.empty((B, n + 1, n + 1), device="cuda"))
        ctrs.append(torch.zeros(1, dtype=torch.int64, device="cuda"))
        starts.append(None)
        if n == L.N_SUB and not args.no_cnn:
            net = fwr.CNN(n, 2 * n, I.pupil_mask(n), max_batch=B, input_scale=L.INPUT_SCALE)
            net.set_params(np.load(os.path.join(ROOT, "paper_1705_04298_amd", "weights",
                                                "cnn_40x40_fried.npz"))["params"])
            starts[-1] = torch.empty((B, 2, 2 * n, 2 * n), device="cuda")
    work = [(p, x, o, s, None) for p, x, o, s in zip(plans, xs, outs, starts)]
    # with the network, its frames (network, then their loop) form a branch of their own on a
    # second stream, beside the grouped loops of the other sizes
    learned = [w for w in work if w[3] is not None]
    others = [w for w in work if w[3] is None]
    branch = torch.cuda.Stream()

    def step():
        for p, x, c in zip(plans, xs, ctrs):
            p.generate(x.shape[0], seed, counter=c, slopes=x, r0=0.15, L0=25.0, sigma=0.05)
        if net is None:
            fwr.reconstruct_group(work)
            return
        main = torch.cuda.current_stream()
        branch.wait_stream(main)
        with torch.cuda.stream(branch):
            net.set_stream()
            for p, x, o, s, _ in learned:
                p.set_stream()
                net.forward(x, s)
                p.reconstruct(x, o, start=s)
        net.set_stream()
        for p, _, _, _, _ in learned:
            p.set_stream()
        fwr.reconstruct_group(others)
        main.wait_stream(branch)

    def rebind():
        for p in plans:
            p.set_stream()
        if net is not None:
            net.set_stream()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rebind()
        for _ in range(2):
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    # eager steps (one stream, launches from Python) for comparison
    rebind()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        step()
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / 20
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rebind()
        step()
    rebind()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    K = args.graph_steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    ev[0].record()
    for k in range(K):
        g.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])
    total_ms = ev[0].elapsed_time(ev[K])
    frames = sum(B for _, B, _ in UNEVEN)
    line = {
        "metric": "frames/s, uneven mixed-size closed loop (10 Gerchberg iters, graph-captured steps)",
        "value": frames * K / (total_ms / 1e3), "unit": "frames/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": total_ms / K, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic (device generator, fresh frames every step)",
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "mean": float(lat.mean())},
        "eager_ms_per_step": eager_ms,
        "config": {"workload": "2048x24^2 + 2048x40^2 (CNN start) + 512x64^2 + 64x128^2 SH frames, padded 2x, "
                               "10 iterations + Eq.5 + MMSE, fresh von Karman frames each step",
                   # (a multi-pass item of the grouped call runs one launch per pass whatever its
                   # tuned schedule: schedule 2's waiting workgroups would hold CUs the others need)
                   "items": [{"n_sub": n, "frames": B, "frames_per_group": p.launch_info()[1],
                              "fft_radix_schedule": p.schedule,
                              **({"loop_in_group": "one launch per pass"} if 2 * n == 256 else {})}
                             for (n, B, _), p in zip(UNEVEN, plans)],
                   "learned_start": net is not None},
    }
    for p in plans:
        p.close()
    if net is not None:
        net.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
