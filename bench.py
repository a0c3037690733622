"""Benchmark of the online LRBMS step (Alg. 3 step 5) on one MI355X.

A step = one pass of the whole online path over one simulation state:
mobility + reduced assembly, reduced solve, pressure/flux reconstruction,
saturation step + limiter, all through the C ABI of liblrbms.so, inputs
resident in HBM.  Prints one JSON line (see the keys below).

Default workload: 2D 256x256 fine cells, 16x16 coarse boxes, log-normal
permeability (corr. length 0.05, sigma_logk 2), Corey exponents 2, viscosity
ratio 5, local bases of size <= 25, FP64, plain per-simulation path.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_model(p, n_snap, cap, seed):
    """Local bases by Gram-Schmidt of seeded smooth snapshot fields (the
    library's own host Gram-Schmidt), N_E = cap in every box."""
    from synth import smooth_fields
    from paper_1405_2810_amd.lrbms import Model
    snaps = smooth_fields(p, n_snap, np.random.default_rng(seed))
    return Model.from_snapshots(p, snaps, ne_cap=cap, unit_functions=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--mode", default="direct", choices=["direct", "affine"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from synth import make_problem, random_saturation
    from paper_1405_2810_amd.lrbms import DIRECT, AFFINE

    p = make_problem(args.config)
    r = p.dim + 1
    log(f"[bench] config {args.config}: building model")
    t0 = time.time()
    gm = build_model(p, n_snap=p.ne_cap + 4, cap=p.ne_cap, seed=p.seed + 1)
    info = gm.info
    log(f"[bench] model ready in {time.time() - t0:.1f}s: N={info['N']} boxes={info['n_sub']} "
        f"device MB={info['device_bytes'] / 1e6:.1f}")
    mode = DIRECT if args.mode == "direct" else AFFINE
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    s0 = torch.as_tensor(random_saturation(p, np.random.default_rng(1), lo=0.0, hi=0.6),
                         dtype=torch.float64, device=dev)
    s_a = s0.clone()
    s_b = torch.zeros_like(s_a)
    pN = torch.zeros(info["N"], dtype=torch.float64, device=dev)
    flux = torch.zeros(info["nface"], dtype=torch.float64, device=dev)
    flags = torch.zeros(info["ncell"], dtype=torch.uint8, device=dev)

    def step(sa, sb, ev=None):
        if ev:
            ev[0].record(st)
        gm.assemble(sa, mode, st)
        if ev:
            ev[1].record(st)
        gm.solve(pN, st)
        if ev:
            ev[2].record(st)
        gm.reconstruct_flux(pN, sa, flux, None, st)
        if ev:
            ev[3].record(st)
        gm.transport_step(sa, flux, sb, flags, st)
        if ev:
            ev[4].record(st)

    for i in range(args.warmup):
        step(s_a, s_b)
        s_a, s_b = s_b, s_a
    torch.cuda.synchronize()
    if gm.status() != 0:
        raise RuntimeError("device status error during warm-up")
    # timed region: K whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(s_a, s_b)
        s_a, s_b = s_b, s_a
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = wall / args.steps * 1e3
    # per-call durations and per-step latency with events on the same stream
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    for i in range(args.steps):
        step(s_a, s_b, evs[i])
        s_a, s_b = s_b, s_a
    torch.cuda.synchronize()
    parts = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(4)] for e in evs])
    lat = parts.sum(axis=1)
    log(f"[bench] step {ms:.3f} ms; per call (ms) assemble {parts[:, 0].mean():.4f} "
        f"solve {parts[:, 1].mean():.4f} flux {parts[:, 2].mean():.4f} "
        f"transport {parts[:, 3].mean():.4f}")
    # transport roofline: algorithmic bytes per launch pair (Euler + limiter)
    nc, nf = info["ncell"], info["nface"]
    tr_bytes = 8 * (2 * r * nc + nf + 2 * nc) + 8 * (2 * r * nc + nf) + nc
    tr_ms = parts[:, 3].mean()
    achieved = tr_bytes / (tr_ms * 1e-3) / 1e9
    out = {
        "metric": "online pressure solves/s + p50/p99 latency vs plain GPU path at rel err<=1e-10",
        "value": 1e3 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: 2D {p.n[0]}x{p.n[1]} fine cells, "
                               f"{len(p.cuts[0]) - 1}x{len(p.cuts[1]) - 1} coarse boxes, "
                               f"N_E<={p.ne_cap}, online step a1-a7, plain per-simulation path",
                   "mode": args.mode, "N": info["N"]},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "per_call_ms": {"assemble": float(parts[:, 0].mean()), "solve": float(parts[:, 1].mean()),
                        "flux": float(parts[:, 2].mean()), "transport": float(parts[:, 3].mean())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "transport_step (k_transport + k_limiter)"},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
