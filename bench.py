"""Benchmark of the online LRBMS step (Alg. 3 step 5) on one MI355X.

A step = one pass of the whole online path over one simulation state:
mobility + reduced assembly, reduced solve, pressure/flux reconstruction,
saturation step + limiter, all through the C ABI of liblrbms.so, inputs
resident in HBM.  Prints one JSON line on stdout (progress goes to stderr).

Default workload: 3D 60x220x85 fine cells (1.12 M) on 600x2200x170 m,
6x22x5 coarse boxes of 10x10x17 cells, layered log-normal permeability
(sigma_logk 3) with seeded high-permeability channels, Corey exponents 2,
viscosity ratio 10, five-spot wells, local bases of size 40 (1_E plus
Gram-Schmidt of seeded smooth snapshot fields), N = 26,400, FP64, the plain
per-simulation path (sequential launches on one stream, no graph, no
batching).  The autotuner (untimed set-up) picks the reduced solver's shapes
and keeps one refinement step in every reduced solve unless the unrefined
solve's own error, measured on the device, is below 1e-13.  The 2D 256x256
workload (16x16 boxes, N_E = 25) is timed after it for context.

Passes, in order:
  warm-up      W untimed steps;
  timed        K steps between two device synchronizations: `value`,
               `ms_per_step`;
  latency      K steps with HIP events between the four calls: p50/p99 step
               latency and the mean time of each call;
  kernels      K steps with the library's per-kernel event timing switched on:
               per kernel kind the mean launch time and the algorithmic
               flops and bytes, hence the roofline of the dominant kernel;
  context      the fine reference (Alg. 1 on the GPU, --fine-steps steps) and
               one run of the GPU offline stage (--offline), reported beside
               the metric;
  extra        the plain path on the --extra-config workload;
  cpu_baseline the GPU's reduced solve against the oracle's solve of the same
               system, then the FP64 CPU oracle's online step on a bounded
               sample of the same workload at all cores and at one thread
               (skipped with --no-cpu-baseline).
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

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector (= FP64 matrix) peak

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record of this kernel and workload, if the kernel's source is unchanged
    since the counters were taken; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from paper_1405_2810_amd.profiling import source_sha
    e = rec.get(workload, {}).get(kernel)
    if not e or e.get("source_sha") != source_sha(kernel):
        return None
    return float(e["bytes_per_launch"])


def build_model(p, n_snap, cap, seed):
    """Local bases by the library's device Gram-Schmidt of seeded smooth
    snapshot fields, 1_E first, N_E = cap in every box."""
    from synth import smooth_fields
    from paper_1405_2810_amd.lrbms import Model
    snaps = smooth_fields(p, n_snap, np.random.default_rng(seed))
    return Model.from_snapshots(p, snaps, ne_cap=cap, unit_functions=True), snaps


def build_ensemble(n: int, seed: int = 500, tune: bool = True):
    """n simulations, alternately 2D 256x256 and 3D 64x64x32 on seeded uneven
    coarse partitions, each with its own permeability seed and seeded local
    basis sizes in 5..60 per box (the first N_E functions of a Gram-Schmidt
    basis of 61 seeded plane-wave fields plus 1_E, shared per grid); tune:
    each member's assembly variant and solver shapes by the autotuner on a
    seeded state of its own."""
    from synth import CONFIGS, make_problem, wave_fields, ensemble_caps
    from paper_1405_2810_amd.lrbms import Model
    snaps, out = {}, []
    for i in range(n):
        name = "ens2d" if i % 2 == 0 else "ens3d"
        p = make_problem(name, seed=CONFIGS[name]["seed"] + i)
        if name not in snaps:
            snaps[name] = wave_fields(p, 61, np.random.default_rng(seed + len(snaps)))
        full = Model.from_snapshots(p, snaps[name], ne_cap=60, unit_functions=True)
        m = full.truncated(ensemble_caps(p, np.random.default_rng(seed + 1000 + i)))
        full.close()
        if tune:
            import torch
            from synth import random_saturation
            s = torch.as_tensor(random_saturation(p, np.random.default_rng(seed + 2000 + i),
                                                  lo=0.0, hi=0.6),
                                dtype=torch.float64, device="cuda")
            m.tuned = m.autotune(s, reps=3)
        out.append((p, m))
    return out


def build_serving_mix(n64: int, n256: int, big=None, seed: int = 600):
    """The serving mix: n64 simulations on the 64x64 grid (4x4 boxes, N_E <= 10)
    and n256 on the 256x256 grid (16x16 boxes, N_E <= 25), each with its own
    permeability seed; the local bases of a grid are one Gram-Schmidt basis of
    seeded smooth snapshot fields of that grid (shared by its simulations);
    big: an existing (problem, model) pair appended to the mix."""
    from synth import CONFIGS, make_problem, smooth_fields
    from paper_1405_2810_amd.lrbms import Model
    out = []
    for name, n in (("cfg1", n64), ("cfg2", n256)):
        if n <= 0:
            continue
        p0 = make_problem(name)
        snaps = smooth_fields(p0, p0.ne_cap + 4, np.random.default_rng(seed))
        base = Model.from_snapshots(p0, snaps, ne_cap=p0.ne_cap, unit_functions=True)
        sizes, flat = base.export_basis()
        base.close()
        for i in range(n):
            p = make_problem(name, seed=CONFIGS[name]["seed"] + 1 + i)
            out.append((p, Model.create(p, sizes, flat)))
    if big is not None:
        out.append(big)
    return out


def _states(members, seed):
    import torch
    from synth import random_saturation
    return [torch.as_tensor(random_saturation(p, np.random.default_rng(seed + i), lo=0.0, hi=0.6),
                            dtype=torch.float64, device="cuda") for i, (p, _) in enumerate(members)]


def bench_batch(members, steps: int, warmup: int):
    """One ensemble step = one online step (DIRECT) of every member.  The
    plain per-simulation path (members one after another on one stream)
    against the batch: members on branches of their own with direct launches
    or captured into one graph (one launch per ensemble step), each with the
    members' own reduced solves or with one fused solve for all members."""
    import torch
    from paper_1405_2810_amd.lrbms import Batch, DIRECT
    st = torch.cuda.current_stream()
    models = [m for _, m in members]
    sats = _states(members, 900)
    bufs = [(torch.zeros(m.info["N"], dtype=torch.float64, device="cuda"),
             torch.zeros(m.info["nface"], dtype=torch.float64, device="cuda"),
             torch.zeros_like(s)) for m, s in zip(models, sats)]

    def plain():
        for m, s, (pN, fl, nx) in zip(models, sats, bufs):
            m.assemble(s, DIRECT, st)
            m.solve(pN, st)
            m.reconstruct_flux(pN, s, fl, None, st)
            m.transport_step(s, fl, nx, None, st)
            s.copy_(nx)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(st)
        for k in range(steps):
            fn()
            ev[k + 1].record(st)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps * 1e3
        lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        return {"ms_per_ensemble_step": wall, "solves_per_s": len(models) * 1e3 / wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}

    res = {"plain": timed(plain)}
    for key, graph, fused in (("batched_streams", False, False), ("batched_graph", True, False),
                              ("fused_solve_streams", False, True),
                              ("fused_solve_graph", True, True)):
        B = Batch(models, mode=DIRECT, graph=graph, fused=fused)
        res[key] = timed(lambda: B.step(sats, None, st))
        if B.status() < 0:
            raise RuntimeError(f"device status error in the {key} pass")
        B.close()
    for m in models:
        if m.status() < 0:
            raise RuntimeError("device status error in the batched pass")
    for k in res:
        res[k]["vs_plain"] = res[k]["solves_per_s"] / res["plain"]["solves_per_s"]
    return res


def bench_serve(members, rates, n_req: int, slots: int, seed: int = 77, fused: bool = False,
                label: str = ""):
    """Poisson arrivals of online-step requests, each for a uniformly drawn
    member, at each rate (rate 0: every request submitted at once, which
    measures the capacity); the server admits every member (the budget is the
    sum of their footprints) and dispatches onto `slots` slot streams;
    slots=1 is the plain path (one request on the device at a time); fused:
    waves of up to `slots` requests whose reduced solves run as one
    combined-plan solve.  Per rate: achieved solves/s (requests over the time
    from the first submit to the last completion) and p50/p99 latency
    (submit to completion seen by poll)."""
    from paper_1405_2810_amd.lrbms import Server, DIRECT
    models = [m for _, m in members]
    sats = _states(members, 700)
    foot = sum(m.info["device_bytes"] + 8 * (m.info["N"] + m.info["nface"] +
                                             m.info["r"] * m.info["ncell"]) for m in models)
    out = {}
    for rate in rates:
        rng = np.random.default_rng(seed)
        arrive = (np.zeros(n_req) if rate <= 0 else
                  np.cumsum(rng.exponential(1.0 / rate, n_req)))
        who = rng.integers(0, len(models), n_req)
        S = Server(hbm_budget=foot, max_slots=slots, mode=DIRECT, fused=fused)
        ids = [S.attach(m, s) for m, s in zip(models, sats)]
        S.poll(0)  # admits the attached simulations
        if S.info()["n_admitted"] != len(models):
            info = S.info()
            S.close()
            raise RuntimeError(f"budget {foot} B did not admit every member: {info}")
        lat = []
        t0 = time.perf_counter()
        k = 0
        last = t0
        while len(lat) < n_req:
            now = time.perf_counter() - t0
            while k < n_req and arrive[k] <= now:
                S.submit(ids[who[k]], k)
                k += 1
            for _, ms, rc in S.poll(1024):
                if rc != 0:
                    raise RuntimeError(f"request failed with status {rc}")
                lat.append(ms)
                last = time.perf_counter()
            if k == n_req and time.perf_counter() - last > 60.0:
                info = S.info()
                S.close()
                raise RuntimeError(f"serving made no progress for 60 s ({len(lat)} of {n_req} "
                                   f"done; server {info})")
        span = time.perf_counter() - t0
        S.close()
        lat = np.array(lat)
        key = "burst" if rate <= 0 else f"{rate:g}"
        out[key] = {"solves_per_s": n_req / span, "p50_ms": float(np.percentile(lat, 50)),
                    "p99_ms": float(np.percentile(lat, 99))}
        log(f"[bench] serve {label} slots={slots}{' fused' if fused else ''} "
            f"{'burst' if rate <= 0 else f'rate {rate:g}/s'}: {n_req / span:.0f} solves/s, "
            f"p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms")
    for m in models:
        if m.status() < 0:
            raise RuntimeError("device status error in the serving pass")
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(p, snaps, s0, n_steps: int, threads: int):
    """Seconds per online step of the oracle (DIRECT, a1-a7; bases built by
    the oracle from the same snapshots, untimed) over n_steps from s0, with
    the BLAS/OpenMP pools limited to `threads`."""
    from threadpoolctl import threadpool_limits
    from oracle.fem import Grid
    from oracle.offline import local_bases
    from oracle.online import Model as OModel, online_step, DIRECT as O_DIRECT
    g = Grid(p)
    phis = local_bases(g, p, snaps, method="gs", cap=p.ne_cap, unit=True)
    om = OModel(p, phis, None)
    s = np.asarray(s0, dtype=np.float64).copy()
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        for _ in range(n_steps):
            s = online_step(om, s, O_DIRECT)["s"]
        return (time.perf_counter() - t0) / n_steps


def cpu_baseline(name: str, p, snaps, s0, n_steps: int):
    """The FP64 CPU oracle's online step timed on the host, at all cores and
    at one thread.  The 3D 60x220x85 workload takes minutes per oracle step,
    so its sample is the same recipe on a slab of 2 of its 22 box rows
    (60x20x85 cells, 6x2x5 boxes of 10x10x17 cells, N_E = 40, the five-spot
    wells of the slab), one step, scaled by the ratio of boxes (660 / 60)."""
    from synth import make_problem, random_saturation, smooth_fields
    ncores = os.cpu_count() or 1
    scale, what = 1.0, f"{n_steps} consecutive online steps of the same workload from the same state"
    if name == "cfg3":
        p = make_problem("cfg3", n=(60, 20, 85), L=(600.0, 200.0, 170.0), nc=(6, 2, 5))
        snaps = smooth_fields(p, p.ne_cap + 4, np.random.default_rng(p.seed + 1))
        s0 = random_saturation(p, np.random.default_rng(1), lo=0.0, hi=0.6)
        n_steps, scale = 1, 660.0 / 60.0
        what = ("one online step of a 2-of-22-box-row slab of the workload (60x20x85 cells, "
                "6x2x5 boxes, N_E = 40, same recipe), scaled by 660/60 boxes")
    t_all = _oracle_steps(p, snaps, s0, n_steps, ncores) * scale
    t_one = _oracle_steps(p, snaps, s0, n_steps, 1) * scale
    return {"value": 1.0 / t_all, "unit": "solves/s", "cores": int(ncores), "kind": "oracle",
            "one_thread": {"value": 1.0 / t_one, "unit": "solves/s", "cores": 1},
            "cpu_model": cpu_model(),
            "sample": f"{what} (DIRECT, a1-a7, FP64 NumPy/SciPy oracle; bases built untimed); "
                      f"{t_all:.1f} s per full-workload step at {ncores} threads, {t_one:.1f} s at "
                      f"1 thread; CPU: {cpu_model()}"}


def solver_parity(gm, sat, mode):
    """Relative L2 distance of the GPU's p_N (after its refinement) from the
    oracle's solve of the same reduced system (the GPU's own A_N, f_N)."""
    import torch
    from oracle.online import solve_reduced
    gm.assemble(sat, mode)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    gm.solve(pN)
    blocks, f = gm.reduced_system()
    x = solve_reduced(gm.sparse_reduced_matrix(blocks, lower=True), f)
    got = pN.cpu().numpy()
    return float(np.linalg.norm(got - x) / np.linalg.norm(x))


def measure_plain(name: str, steps: int, warmup: int, autotune: int):
    """The plain per-simulation path on another workload: ms per online step."""
    import torch
    from synth import make_problem, random_saturation
    from paper_1405_2810_amd.lrbms import DIRECT
    p = make_problem(name)
    gm, _ = build_model(p, n_snap=p.ne_cap + 4, cap=p.ne_cap, seed=p.seed + 1)
    st = torch.cuda.current_stream()
    s_a = torch.as_tensor(random_saturation(p, np.random.default_rng(1), lo=0.0, hi=0.6),
                          dtype=torch.float64, device="cuda")
    tune = gm.autotune(s_a, reps=10) if autotune else None
    s_b = torch.zeros_like(s_a)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    flux = torch.zeros(gm.info["nface"], dtype=torch.float64, device="cuda")
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        gm.assemble(s_a, DIRECT, st)
        gm.solve(pN, st)
        gm.reconstruct_flux(pN, s_a, flux, None, st)
        gm.transport_step(s_a, flux, s_b, None, st)
        s_a, s_b = s_b, s_a
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    status = gm.status()
    info = gm.info
    gm.close()
    if status < 0:
        raise RuntimeError(f"device status error on {name}")
    nc = [len(c) - 1 for c in p.cuts[:p.dim]]
    log(f"[bench] {name}: {ms:.3f} ms/step ({1e3 / ms:.0f} solves/s)")
    return {"workload": f"{name}: {p.dim}D {'x'.join(str(v) for v in p.n[:p.dim])} fine cells, "
                        f"{'x'.join(str(v) for v in nc)} coarse boxes, N_E<={p.ne_cap}, plain path",
            "N": info["N"], "ms_per_step": ms, "solves_per_s": 1e3 / ms, "solver_shapes": tune,
            "cfl_warning": status == 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cfg3")
    ap.add_argument("--extra-config", default="cfg2",
                    help="a second workload timed on the plain path for context ('' skips)")
    ap.add_argument("--mode", default="direct", choices=["direct"])
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fine-steps", type=int, default=3,
                    help="steps of the fine reference (Alg. 1) timed for context; 0 skips")
    ap.add_argument("--offline", type=int, default=-1,
                    help="1: time the GPU offline stage once for context (-1: only for 2D "
                         "workloads; the 3D one takes about a minute)")
    ap.add_argument("--ensemble", type=int, default=64,
                    help="members of the batched ensemble pass; 0 skips it")
    ap.add_argument("--ensemble-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=1500,
                    help="requests per rate of the serving pass; 0 skips it")
    ap.add_argument("--serve-64", type=int, default=128,
                    help="simulations on the 64x64 grid in the serving mix")
    ap.add_argument("--serve-256", type=int, default=96,
                    help="simulations on the 256x256 grid in the serving mix")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: pick the reduced solver's shapes by timing them (untimed set-up)")
    ap.add_argument("--shapes", default="",
                    help="leaf,split,bw[,asm]: install these solver shapes (0 = never split) and "
                         "box-assembly variant instead of autotuning, e.g. to profile the "
                         "configuration a timed run chose")
    ap.add_argument("--refine", type=int, default=-1,
                    help=">= 0: refinement steps of the reduced solve, set after the autotuner")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 256 MiB (scale of the HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = (256 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): the online step of one "
              "simulation runs on one device and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from synth import make_problem, random_saturation
    from paper_1405_2810_amd.lrbms import DIRECT, AFFINE

    p = make_problem(args.config)
    if args.offline < 0:
        args.offline = 1 if p.dim == 2 else 0
    r = p.dim + 1
    log(f"[bench] config {args.config}: building model")
    t0 = time.time()
    gm, snaps = build_model(p, n_snap=p.ne_cap + 4, cap=p.ne_cap, seed=p.seed + 1)
    info = gm.info
    log(f"[bench] model ready in {time.time() - t0:.1f}s: N={info['N']} boxes={info['n_sub']} "
        f"device MB={info['device_bytes'] / 1e6:.1f}")
    mode = DIRECT if args.mode == "direct" else AFFINE
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    s0_host = random_saturation(p, np.random.default_rng(1), lo=0.0, hi=0.6)
    s0 = torch.as_tensor(s0_host, dtype=torch.float64, device=dev)
    tune = gm.autotune(s0, reps=10) if args.autotune and not args.shapes else None
    if args.shapes:
        vals = [int(v) for v in args.shapes.split(",")]
        leaf, split, bw = vals[:3]
        asm = vals[3] if len(vals) > 3 else 0
        gm.set_solver_shapes(leaf, split, bw)
        gm.set_assembly_variant(asm)
        log(f"[bench] shapes set: leaf {leaf} split {split} backward split {bw}, assembly "
            f"variant {asm}")
        shapes = dict(leaf_max=leaf, split_min=split, bw_split_min=bw, asm_variant=asm,
                      source="--shapes")
    else:
        shapes = tune
    if tune:
        log(f"[bench] assembly autotune: variant {tune['asm_variant']} "
            f"({tune['asm_us'][0]:.1f} / {tune['asm_us'][1]:.1f} us per assembly)")
        log(f"[bench] solver autotune: leaf {tune['leaf_max']} split {tune['split_min']} "
            f"backward split {tune['bw_split_min']}, unrefined error "
            f"{tune['unrefined_error']:.1e} -> refinement steps {tune['refine']}: "
            f"{tune['us_per_solve']:.1f} us per solve (was {tune['us_before']:.1f}, "
            f"{tune['n_candidates']} shapes)")
    refine_steps = tune["refine"] if tune else 1
    if args.refine >= 0:
        gm.set_refinement(args.refine)
        refine_steps = args.refine
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
    if gm.status() < 0:
        raise RuntimeError("device status error during warm-up")
    log(f"[bench] warm-up done ({args.warmup} steps); timing {args.steps} steps")
    # ---- timed region: K whole steps -------------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(s_a, s_b)
        s_a, s_b = s_b, s_a
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = wall / args.steps * 1e3
    status = gm.status()
    if status < 0:
        raise RuntimeError("device status error in the timed region")
    cfl_warning = status == 1
    log(f"[bench] timed: {ms:.3f} ms/step")
    # ---- latency pass ------------------------------------------------------
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    for i in range(args.steps):
        step(s_a, s_b, evs[i])
        s_a, s_b = s_b, s_a
    torch.cuda.synchronize()
    parts = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(4)] for e in evs])
    lat = parts.sum(axis=1)
    log(f"[bench] per call (ms) assemble {parts[:, 0].mean():.4f} solve {parts[:, 1].mean():.4f} "
        f"flux {parts[:, 2].mean():.4f} transport {parts[:, 3].mean():.4f}")
    # ---- per-kernel pass ---------------------------------------------------
    gm.profile_enable(True)
    for i in range(args.steps):
        step(s_a, s_b)
        s_a, s_b = s_b, s_a
    kstats = gm.profile_read()
    gm.profile_enable(False)
    kernels = {}
    for name, e in kstats.items():
        avg_ms = e["total_ms"] / e["launches"]
        gbs = e["bytes"] / (e["total_ms"] * 1e-3) / 1e9 if e["total_ms"] > 0 else 0.0
        tfs = e["flops"] / (e["total_ms"] * 1e-3) / 1e12 if e["total_ms"] > 0 else 0.0
        t_hbm = e["bytes"] / (PEAK_HBM_GBS * 1e9)
        t_alu = e["flops"] / (PEAK_FP64_TFLOPS * 1e12)
        kernels[name] = {"launches_per_step": e["launches"] / args.steps,
                         "avg_launch_us": avg_ms * 1e3,
                         "ms_per_step": e["total_ms"] / args.steps,
                         "bytes_per_launch": e["bytes"] / e["launches"],
                         "flops_per_launch": e["flops"] / e["launches"],
                         "GBs": gbs, "TFLOPs": tfs,
                         "bound": "hbm" if t_hbm >= t_alu else "alu"}
    for name, k in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"[bench]   {name:18s} {k['launches_per_step']:5.1f}/step {k['avg_launch_us']:9.2f} us "
            f"{k['ms_per_step']:8.4f} ms/step  {k['GBs']:8.1f} GB/s {k['TFLOPs']:7.3f} TF/s "
            f"({k['bound']})")
    dom = max(kernels, key=lambda n: kernels[n]["ms_per_step"])
    kd = kernels[dom]
    workload = f"{args.config}-{args.mode}"
    traffic = measured_traffic(dom, workload)
    if kd["bound"] == "hbm":
        roof = {"bound": "hbm", "achieved": kd["GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": kd["GBs"] / PEAK_HBM_GBS}
    else:
        roof = {"bound": "alu", "achieved": kd["TFLOPs"], "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": kd["TFLOPs"] / PEAK_FP64_TFLOPS}
    roof["traffic"] = traffic
    roof["kernel"] = dom
    roof["avg_launch_us"] = kd["avg_launch_us"]
    roof["algorithmic_per_launch"] = {"bytes": kd["bytes_per_launch"], "flops": kd["flops_per_launch"]}
    # ---- context: the fine reference (Alg. 1) and the offline stage on the GPU
    extras = {}
    if args.fine_steps > 0:
        from paper_1405_2810_amd.lrbms import Fine
        fine = Fine(p)
        sf_a, sf_b = s0.clone(), torch.zeros_like(s0)
        ph = torch.zeros_like(s0)
        its = []
        fine.step(sf_a, ph, flux, sf_b, flags)          # first solve: hierarchy set-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.fine_steps):
            it, _ = fine.step(sf_a, ph, flux, sf_b, flags, warm=True)
            its.append(it)
            sf_a, sf_b = sf_b, sf_a
        torch.cuda.synchronize()
        fms = (time.perf_counter() - t0) / args.fine_steps * 1e3
        fine.close()
        extras["fine_reference"] = {
            "what": "Alg. 1 on the same GPU: fine SWIP pressure by multigrid-preconditioned CG "
                    "(rtol 1e-13, warm start), fluxes, transport, limiter",
            "ms_per_step": fms, "cg_iterations_mean": float(np.mean(its)),
            "steps": args.fine_steps, "online_speedup": fms / ms}
        log(f"[bench] fine reference: {fms:.2f} ms/step, {np.mean(its):.0f} CG iterations; "
            f"online step is {fms / ms:.1f}x faster")
    if args.offline:
        from synth import training_params
        from paper_1405_2810_amd.lrbms import Model
        params = training_params(p.M, p.n_train, np.random.default_rng(p.seed))
        T = p.t_end if p.t_end > 0 else p.n_steps * p.dt
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        om, rep = Model.build_offline(p, params, ne_cap=p.ne_cap, horizon=T, pcg_rtol=1e-12)
        osec = time.perf_counter() - t0
        extras["offline_stage"] = {"seconds": osec, "N": om.info["N"], **rep}
        om.close()
        log(f"[bench] offline stage (Alg. 2 without greedy) on the GPU: {osec:.2f} s, {rep}")
    if args.ensemble > 0:
        log(f"[bench] ensemble: building {args.ensemble} members")
        t0 = time.time()
        members = build_ensemble(args.ensemble)
        sz = [m.info["N"] for _, m in members]
        log(f"[bench] ensemble ready in {time.time() - t0:.1f}s: N {min(sz)}..{max(sz)}, "
            f"device MB {sum(m.info['device_bytes'] for _, m in members) / 1e6:.0f}")
        bat = bench_batch(members, args.ensemble_steps, 3)
        for k, v in bat.items():
            log(f"[bench] ensemble {k}: {v['ms_per_ensemble_step']:.2f} ms per ensemble step, "
                f"{v['solves_per_s']:.0f} solves/s, p99 {v['p99_ms']:.2f} ms")
        # the same members served (fused waves of up to 64 requests) against the
        # fused batch step
        if args.serve_requests > 0:
            bat["served_fused_waves"] = bench_serve(members, [0, 5e4], args.serve_requests, 64,
                                                    fused=True, label="ensemble")
        tuned = [getattr(m, "tuned", None) for _, m in members]
        tuned_summary = None
        if all(t is not None for t in tuned):
            from collections import Counter
            tuned_summary = {
                "asm_variant": dict(Counter(f"{'2D' if p.dim == 2 else '3D'} variant "
                                            f"{t['asm_variant']}" for (p, _), t in
                                            zip(members, tuned))),
                "leaf_max": dict(Counter(str(t["leaf_max"]) for t in tuned)),
                "refine": dict(Counter(str(t["refine"]) for t in tuned))}
            log(f"[bench] ensemble tuned shapes: {tuned_summary}")
        bat["tuned_shapes"] = tuned_summary
        extras["ensemble"] = {
            "what": f"{args.ensemble} simulations, alternately 2D 256x256 and 3D 64x64x32 on "
                    "seeded uneven coarse partitions, seeded N_E in 5..60 per box, DIRECT online "
                    "step per member; served_fused_waves: the same members behind the server "
                    "(Poisson arrivals, uniformly drawn members, 'burst' = all at once)",
            "members": args.ensemble, "N_range": [min(sz), max(sz)], **bat}
        for _, m in members:
            m.close()
    if args.serve_requests > 0:
        log(f"[bench] serving mix: building {args.serve_64} x 64x64 and {args.serve_256} x "
            f"256x256 simulations, plus the {args.config} model")
        t0 = time.time()
        mix = build_serving_mix(args.serve_64, args.serve_256, big=(p, gm))
        log(f"[bench] serving mix ready in {time.time() - t0:.1f}s: {len(mix)} simulations, "
            f"device MB {sum(m.info['device_bytes'] for _, m in mix) / 1e6:.0f}")
        rates = [0, 1e3, 1e4, 5e4]
        nreq = args.serve_requests
        serve = {"continuous": bench_serve(mix, rates, nreq, args.serve_slots, label="mix"),
                 "fused_waves": bench_serve(mix, rates, nreq, 64, fused=True, label="mix"),
                 "plain_one_slot": bench_serve(mix, rates, nreq, 1, label="mix")}
        caps = {k: max(r["solves_per_s"] for r in v.values()) for k, v in serve.items()}
        best = max(caps, key=caps.get)
        cap = caps[best]
        below = 0.8 * cap
        serve[best][f"{below:.0f} (0.8 capacity)"] = bench_serve(
            mix, [below], nreq, 64 if best == "fused_waves" else
            (1 if best == "plain_one_slot" else args.serve_slots),
            fused=best == "fused_waves", label="mix")[f"{below:g}"]
        extras["serving"] = {
            "what": f"{len(mix)} concurrent simulations: {args.serve_64} on 64x64 (4x4 boxes, "
                    f"N_E <= 10), {args.serve_256} on 256x256 (16x16 boxes, N_E <= 25), each with "
                    f"its own permeability seed, and the {args.config} model; Poisson arrivals "
                    f"of single online-step requests for uniformly drawn simulations, {nreq} "
                    "requests per rate ('burst': all at once, the capacity); continuous: "
                    f"{args.serve_slots} slot streams; fused_waves: waves of up to 64 requests "
                    "with one combined-plan reduced solve; plain_one_slot: one request on the "
                    "device at a time (the plain per-simulation path)",
            "simulations": len(mix), "capacity_solves_per_s": caps, "best": best, **serve}
        for q, m in mix:
            if m is not gm:
                m.close()
    if args.extra_config:
        extras[args.extra_config] = measure_plain(args.extra_config, args.steps, args.warmup,
                                                  args.autotune)
    # ---- CPU oracle baseline, and the GPU solve against the oracle's ------
    cpu, parity = None, None
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        log("[bench] solver parity: the oracle's solve of the GPU's own reduced system")
        parity = {"pN_rel_l2_vs_oracle_solve_of_same_system": solver_parity(gm, s0, mode),
                  "refinement_steps": refine_steps,
                  "unrefined_error_measured": tune["unrefined_error"] if tune else None,
                  "note": "A_N/f_N parity with the oracle's own assembly and the end-to-end "
                          "p_N bound (1e-10) are tested on the 256x256 workload and on the 3D "
                          "workload's coarse grid at 30x110x40 (tests/gpu/test_fullsize.py)"}
        log(f"[bench] solver parity {parity['pN_rel_l2_vs_oracle_solve_of_same_system']:.2e}")
        log(f"[bench] cpu baseline: oracle ({args.config})")
        cpu = cpu_baseline(args.config, p, snaps, s0_host, args.cpu_steps)
        log(f"[bench] cpu baseline: {cpu['value']:.4f} solves/s on {cpu['cores']} threads, "
            f"{cpu['one_thread']['value']:.4f} on 1 ({cpu['cpu_model']})")
    nc = [len(c) - 1 for c in p.cuts[:p.dim]]
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
        "config": {"workload": f"{args.config}: {p.dim}D "
                               f"{'x'.join(str(v) for v in p.n[:p.dim])} fine cells, "
                               f"{'x'.join(str(v) for v in nc)} coarse boxes, N_E<={p.ne_cap}, "
                               f"online step a1-a7 ({args.mode}), plain per-simulation path",
                   "mode": args.mode, "N": info["N"], "fine_cells": info["ncell"],
                   "solver_shapes": shapes},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "per_call_ms": {"assemble": float(parts[:, 0].mean()), "solve": float(parts[:, 1].mean()),
                        "flux": float(parts[:, 2].mean()), "transport": float(parts[:, 3].mean())},
        "pressure_solves_per_s": 1e3 / float((parts[:, 0] + parts[:, 1]).mean()),
        "roofline": roof,
        "parity": parity,
        "cfl_warning": cfl_warning,
        "kernels": {k: {"avg_launch_us": round(v["avg_launch_us"], 3),
                        "launches_per_step": v["launches_per_step"],
                        "GBs": round(v["GBs"], 2), "TFLOPs": round(v["TFLOPs"], 4)}
                    for k, v in kernels.items()},
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
