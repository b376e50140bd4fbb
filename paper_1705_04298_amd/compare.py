"""Extension methods compared on the same synthetic frames (Sec. 4.1): zero padding, the
Hudgin extension, and the Gerchberg extension with and without Eq. 5 at several iteration
counts.  Error = median over frames of the rms phase error on the pupil nodes (piston removed)
against the true screen; every reconstruction runs in libfwr.  `--model sinc` takes frames
measured by the lenslet-averaging model of Eq. 4 and reconstructs with that model.

    python -m paper_1705_04298_amd.compare --frames 4096 [--model sinc]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys

import numpy as np

from . import fwr
from . import inputs as I

N_SUB, N_GRID = 40, 80


WORKLOADS = {"fried": I.SPHERE_40, "sinc": I.SPHERE_40_SINC}


def _chunk(args):
    start, count, model = args
    s = np.empty((count, 2, N_SUB, N_SUB), dtype=np.float32)
    p = np.empty((count, N_SUB + 1, N_SUB + 1))
    for i in range(count):
        s[i], p[i] = I.make_frame(WORKLOADS[model], start + i)
    return s, p


def frames(count: int, start: int = 20_000, workers: int = 0, model: str = "fried"):
    """SPHERE-like 40x40 frames with their true node phase."""
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(start + i, min(64, count - i), model) for i in range(0, count, 64)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_chunk, jobs)
    return np.concatenate([a for a, _ in parts]), np.concatenate([b for _, b in parts])


def compare(count: int = 4096, iters=(1, 2, 3, 5, 10, 20, 50), log=print, model: str = "fried"):
    import torch
    slopes, truth = frames(count, model=model)
    mask = I.pupil_mask(N_SUB)
    nodes = I.pupil_nodes(mask)
    x = torch.from_numpy(slopes).cuda()

    def err(phase):
        e = (phase.cpu().numpy() - truth)[:, nodes]
        e = e - e.mean(axis=1, keepdims=True)
        return float(np.median(np.sqrt(np.mean(e * e, axis=1))))

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = []

    def add(method, k, periodic, phase, ms):
        rows.append({"method": method, "n_iter": k, "periodic": periodic, "median_err_rad": err(phase),
                     "ms_per_batch": ms})
        log(f"[compare] {method:10s} it={k:3d} periodic={periodic}: error {rows[-1]['median_err_rad']:.4f} rad, "
            f"{ms:.3f} ms / {count} frames")

    for periodic in (False, True):
        plan = fwr.Plan(N_SUB, N_GRID, mask, n_iter=0, periodic=periodic, max_batch=count, model=model)
        add("zero-pad", 0, periodic, plan.reconstruct(x), timed(lambda: plan.reconstruct(x)))
        plan.close()
    plan0 = fwr.Plan(N_SUB, N_GRID, mask, n_iter=0, periodic=False, max_batch=count, model=model)
    ext = plan0.hudgin_extend(x)
    add("hudgin", 0, True, plan0.reconstruct(x, start=ext),
        timed(lambda: (plan0.hudgin_extend(x, ext), plan0.reconstruct(x, start=ext))))
    plan0.close()
    for periodic in (False, True):
        for k in iters:
            plan = fwr.Plan(N_SUB, N_GRID, mask, n_iter=k, periodic=periodic, max_batch=count, model=model)
            add("gerchberg", k, periodic, plan.reconstruct(x), timed(lambda: plan.reconstruct(x)))
            plan.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=4096)
    ap.add_argument("--model", choices=sorted(WORKLOADS), default="fried")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    rows = compare(args.frames, log=lambda m: print(m, file=sys.stderr, flush=True), model=args.model)
    print(json.dumps({"frames": args.frames, "model": args.model, "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
