"""Summaries of rocprofv3 output for the kernels of liblrbms.so.

  python -m paper_1405_2810_amd.profiling stats  <kernel_stats.csv> <title> <command> <out.txt>
  python -m paper_1405_2810_amd.profiling traffic <workload> <fetch_dir> <write_dir>
         <calib_fetch_dir> <calib_write_dir> <steps> <out.json> <out.txt> <command...>
  python -m paper_1405_2810_amd.profiling mfma <pmc_dir> <kernel_stats.csv> <title> <out.txt>
         <command...>

`stats` turns a `--kernel-trace --stats` kernel_stats.csv into a short text
table.  `traffic` reads four `--pmc` counter-collection CSVs (FETCH_SIZE and
WRITE_SIZE, each for the benchmark and for a plain device copy of known size),
scales each counter by what it reads for the copy (bytes per KiB counted), and
records per kernel the HBM bytes per launch with the sha256 of the kernel's
source file, so that a figure taken before a change of the kernel is not used.
`mfma` reads one `--pmc SQ_INSTS_VALU_MFMA_MOPS_F64` run: per kernel the FP64
matrix-core flops per launch (MOPS x 512), their rate over the kernel's mean
launch time from a `--kernel-trace --stats` run of the same passes, and that
rate against the FP64 matrix peak.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(path_or_dir: str, pattern: str):
    files = [path_or_dir] if os.path.isfile(path_or_dir) else \
        glob.glob(os.path.join(path_or_dir, "**", pattern), recursive=True)
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def short_name(kernel: str) -> str:
    k = kernel.replace("(anonymous namespace)::", "").split("(")[0].strip()
    for pre in ("void ", "lrbms::"):
        k = k.replace(pre, "")
    return k.split("<")[0].strip()


def stats_table(csv_path: str):
    out = []
    for r in _rows(csv_path, "*kernel_stats.csv"):
        name = r.get("Name") or r.get("KERNEL_NAME") or r.get("Kernel_Name")
        calls = int(r.get("Calls") or r.get("Count") or 0)
        total = float(r.get("TotalDurationNs") or r.get("Total_Duration_ns") or 0)
        avg = float(r.get("AverageNs") or (total / calls if calls else 0))
        pct = float(r.get("Percentage") or 0)
        out.append((name, calls, total, avg, pct))
    out.sort(key=lambda t: -t[2])
    return out


def counters(path: str, counter: str):
    """Per short kernel name: list of counter values (one per dispatch)."""
    vals = {}
    for r in _rows(path, "*counter_collection.csv"):
        if (r.get("Counter_Name") or "").strip() != counter:
            continue
        k = short_name(r.get("Kernel_Name", ""))
        vals.setdefault(k, []).append(float(r["Counter_Value"]))
    return vals


_ASM = ("assemble.hip", "swip.h", "common.h")
_SOLVER = ("solver.hip", "solver.h", "common.h")
_TRANSPORT = ("transport.hip", "common.h")
_OFFLINE = ("offline.hip", "swip.h", "common.h")
_BASES = ("bases.hip", "common.h")
KERNEL_SOURCE = {
    "k_moments": _ASM, "k_lsq": _ASM, "k_lsq_partial": _ASM, "k_lsq_final": _ASM,
    "k_affine_sum": _ASM, "k_asm_box": _ASM, "k_reduce_box": _ASM, "k_asm_iface": _ASM,
    "k_front_asm": _SOLVER, "k_front_factor0": _SOLVER, "k_front_step": _SOLVER,
    "k_front_backward": _SOLVER, "k_front_update": _SOLVER, "k_front_bw_gemv": _SOLVER,
    "k_residual": _SOLVER, "k_front_forward": _SOLVER, "k_front_fw_gemv": _SOLVER,
    "k_front_schur": _SOLVER,
    "k_reconstruct": _TRANSPORT, "k_flux": _TRANSPORT, "k_transport": _TRANSPORT,
    "k_limiter": _TRANSPORT,
    **{k: _OFFLINE for k in ("k_fine_stencil", "k_fine_rhs", "k_fine_jacobi", "k_mg_extract",
                             "k_mg0_down", "k_mg0_up", "k_mgl_down", "k_mgl_up", "k_mg_coarse",
                             "k_power", "k_power_start", "k_cg_init", "k_cg_direction",
                             "k_cg_update", "k_tof_setup", "k_tof_sweep")},
    **{k: _BASES for k in ("k_local_gs", "k_local_pca", "k_basis_compact")},
}


def source_sha(kernel: str) -> str:
    """sha256 (16 hex digits) of the source files a kernel is built from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCE[kernel]:
        with open(os.path.join(ROOT, "paper_1405_2810_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main(argv):
    if argv[0] == "stats":
        csv_path, title, command, out = argv[1:5]
        rows = stats_table(csv_path)
        with open(out, "w") as f:
            f.write(f"# {title}\n# command: {command}\n")
            f.write(f"{'kernel':60s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}\n")
            for name, calls, total, avg, pct in rows:
                f.write(f"{short_name(name)[:60]:60s} {calls:7d} {total / 1e6:10.3f} "
                        f"{avg / 1e3:10.2f} {pct:6.2f}\n")
        print(open(out).read())
        return
    if argv[0] == "traffic":
        workload, fdir, wdir, cfdir, cwdir, steps, out_json, out_txt = argv[1:9]
        command = " ".join(argv[9:])
        steps = int(steps)
        copy_bytes = 256 << 20
        fetch, write = counters(fdir, "FETCH_SIZE"), counters(wdir, "WRITE_SIZE")
        cf, cw = counters(cfdir, "FETCH_SIZE"), counters(cwdir, "WRITE_SIZE")

        def copy_scale(d):
            # the largest dispatches of the calibration run are the 256 MiB copies
            allv = sorted(v for vs in d.values() for v in vs)
            top = allv[-3:]
            return copy_bytes / (sum(top) / len(top))

        sf, sw = copy_scale(cf), copy_scale(cw)
        rec = {}
        if os.path.exists(out_json):
            with open(out_json) as f:
                rec = json.load(f)
        entry = {}
        lines = [f"# HBM traffic per launch, workload {workload}",
                 f"# command: {command}",
                 f"# scale: FETCH_SIZE x {sf:.1f} B, WRITE_SIZE x {sw:.1f} B "
                 f"(plain copy of {copy_bytes} B)",
                 f"{'kernel':24s} {'launches':>8s} {'fetch_MB':>10s} {'write_MB':>10s} {'MB/launch':>10s}"]
        for k in sorted(set(fetch) | set(write)):
            if k not in KERNEL_SOURCE:
                continue
            fv, wv = fetch.get(k, []), write.get(k, [])
            n = max(len(fv), len(wv))
            fb = sum(fv) * sf / max(len(fv), 1)
            wb = sum(wv) * sw / max(len(wv), 1)
            kk = "k_lsq" if k.startswith("k_lsq") else k
            entry[kk] = {"bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb,
                         "write_bytes_per_launch": wb, "launches": n,
                         "source_sha": source_sha(k), "command": command}
            lines.append(f"{k:24s} {n:8d} {fb / 1e6:10.3f} {wb / 1e6:10.3f} {(fb + wb) / 1e6:10.3f}")
        rec[workload] = entry
        with open(out_json, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
        with open(out_txt, "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    if argv[0] == "mfma":
        pmc_dir, stats_csv, title, out = argv[1:5]
        command = " ".join(argv[5:])
        peak = 78.6e12        # FP64 matrix peak of the GPU, FLOP/s
        mops = counters(pmc_dir, "SQ_INSTS_VALU_MFMA_MOPS_F64")
        avg_ns = {}
        for name, calls, total, avg, pct in stats_table(stats_csv):
            k = short_name(name)
            if k in KERNEL_SOURCE and calls:
                avg_ns[k] = avg
        lines = [f"# {title}", f"# command: {command}",
                 "# FP64 matrix flops = SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 per launch; rate over the "
                 "mean launch time of the kernel-stats run; peak 78.6 TFLOP/s",
                 f"{'kernel':20s} {'launches':>8s} {'MFLOP/launch':>13s} {'avg_us':>9s} "
                 f"{'TFLOP/s':>8s} {'of peak':>8s}"]
        for k in sorted(mops):
            if k not in KERNEL_SOURCE:
                continue
            v = mops[k]
            fl = sum(v) * 512.0 / len(v)
            if fl == 0.0:
                continue
            t = avg_ns.get(k, 0.0) * 1e-9
            rate = fl / t if t > 0 else 0.0
            lines.append(f"{k:20s} {len(v):8d} {fl / 1e6:13.2f} {t * 1e6:9.2f} "
                         f"{rate / 1e12:8.3f} {100 * rate / peak:7.2f}%")
        with open(out, "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
