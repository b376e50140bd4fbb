"""Noise propagation of the reconstruction (Sec. 4.1: error propagation coefficient versus
Gerchberg iterations, with and without Eq. 5).

The method is linear in the slopes, so white slope noise alone measures how much noise reaches
the phase.  Coefficient = mean over frames of sum over the pupil nodes of (phi - its mean over
the pupil nodes)^2, divided by (number of pupil nodes x sigma^2): the variance per phase point
per unit slope-noise variance, piston removed.

Frames are noise only: `fwr_generate` with a vanishing turbulence strength (r0 = 1e30 m, so the
screen is below float resolution) and slope noise sigma; every reconstruction runs in libfwr.

    python -m paper_1705_04298_amd.noiseprop --n 40 --frames 4096
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import fwr
from . import inputs as I

NO_TURBULENCE_R0 = 1e30


def coefficient(n: int, N: int, n_iter: int, periodic: bool, frames: int = 4096, sigma: float = 1.0,
                seed: int = 7, d: float | None = None, plan_kwargs=None) -> float:
    """Monte-Carlo noise propagation coefficient of the GPU reconstruction."""
    import torch
    mask = I.pupil_mask(n)
    d = 8.0 / n if d is None else d
    kw = dict(plan_kwargs or {})
    plan = fwr.Plan(n, N, mask, n_iter=n_iter, periodic=periodic, d=d, max_batch=frames, **kw)
    x, _ = plan.generate(frames, seed, r0=NO_TURBULENCE_R0, sigma=sigma)
    phase = plan.reconstruct(x)
    nodes = torch.from_numpy(I.pupil_nodes(mask)).to(phase.device)
    v = phase[:, nodes].double()
    v = v - v.mean(dim=1, keepdim=True)
    c = float((v * v).mean()) / (sigma * sigma)
    plan.close()
    return c


def table(n: int = 40, frames: int = 4096, iters=(0, 1, 2, 3, 5, 10, 20, 50), log=print):
    N = 2 * n
    out = []
    for periodic in (False, True):
        for k in iters:
            c = coefficient(n, N, k, periodic, frames)
            out.append({"n_iter": k, "periodic": periodic, "coefficient": c})
            log(f"[noiseprop] n={n} N={N} it={k:3d} periodic={periodic}: {c:.5f}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=40)
    ap.add_argument("--frames", type=int, default=4096)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    rows = table(args.n, args.frames, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps({"n_sub": args.n, "n_grid": 2 * args.n, "frames": args.frames, "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
