"""Benchmark: FP64 point-Jacobi PCG on one MI355X.

One step is one full solve of the 151 x 301 x 601 bipole workload through
pot3d_solve_device.  The step covers:
* b from Br;
* the initial residual;
* the graph-replayed iterations (p update + A p + p.Ap; r/x update + A p +
  r.z, r.r; two finishers);
* the true residual, the pole values and the copy of Phi out.
Br and Phi are already in HBM; the context (tables and graph) is created
before timing.

  value    = PCG iterations per second over the K timed solves
  roofline = the dominant kernel's algorithmic bytes per launch divided by
             its average launch time (hipEvents, same stream), against
             8 TB/s HBM
  cpu_baseline = the FP64 CPU oracle on the host cores: a bounded number of
             iterations of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels.hip", "solver.hpp"):
        with open(os.path.join(ROOT, "paper_1709_01126_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def summarize_pmc(workload: str, fetch_dir: str, write_dir: str):
    """HBM bytes per launch of the two iteration kernels from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the device copy of N doubles in the same run (known bytes / counter)."""
    import csv
    import glob
    import statistics

    from workloads import WORKLOADS

    n = WORKLOADS[workload].n

    def per_kernel(folder, counter):
        path = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)[0]
        out = {}
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] == counter:
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]) * 1024.0)
        return out

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy_fetch = fetch["__amd_rocclr_copyBuffer"][-1]
    copy_write = write["__amd_rocclr_copyBuffer"][-1]
    f_scale = 8.0 * n / copy_fetch
    w_scale = 8.0 * n / copy_write
    kernels = {}
    for key, mode in (("update_p", ", 2, double>"), ("update_r", ", 3, double>")):
        name = [k for k in fetch if "stencil_" in k and mode in k][0]
        # dispatches that ran (the graph's launches after convergence return at once)
        real_f = [x for x in fetch[name] if x > 0.1 * max(fetch[name])]
        real_w = [x for x in write[name] if x > 0.1 * max(write[name])]
        fb = statistics.median(real_f) * f_scale
        wb = statistics.median(real_w) * w_scale
        alg = (24.0 if key == "update_p" else 40.0) * n
        kernels[key] = {"kernel": name.split("(")[0], "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                        "hbm_bytes_per_launch": fb + wb, "alg_bytes_per_launch": alg,
                        "traffic_over_alg": (fb + wb) / alg}
    out = {"workload": workload, "kernel_source_hash": kernel_source_hash(),
           "calibration": {"copy_bytes": 8.0 * n, "fetch_counter_bytes": copy_fetch, "write_counter_bytes": copy_write,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": kernels}
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def kernel_name(stats, which):
    tile = stats["tile_p"] if which == "update_p" else stats["tile_r"]
    mode = 2 if which == "update_p" else 3
    if tile > 100:
        return f"stencil_wave<{tile - 100},{mode},double>"
    return f"stencil_march<{tile},{mode},double>"


def cpu_baseline(w, faces, br, budget_s: float):
    import oracle

    rf, tf, pf = faces
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br)
    # a warm-up run, a short run to size the sample, then a run of about budget_s seconds
    oracle.pcg(coef, b, 0.0, 1)
    t0 = time.perf_counter()
    oracle.pcg(coef, b, 0.0, 5)
    per = max(1e-3, (time.perf_counter() - t0) / 5)
    k = max(3, int(budget_s / per))
    t0 = time.perf_counter()
    _, iters, _, _ = oracle.pcg(coef, b, 0.0, k)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": iters / dt, "unit": "iter/s", "cores": cores, "kind": "oracle",
            "sample": f"{iters} FP64 Jacobi-PCG iterations of {w.describe()} (tol=0, fixed count), "
                      f"{dt:.1f} s, OpenMP threads={cores}; assembly excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bipole_151x301x601")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders (FETCH_SIZE, WRITE_SIZE) of a --profile-kernels "
                         "run into profiles/traffic_<workload>.json and exit")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="short run for hardware counters: a few iterations, the two stencil kernels "
                         "--kernel-reps times each, and one device copy of N doubles (counter calibration)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.workload, *args.summarize_pmc)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this solver runs on a single device (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_01126_amd import Solver, pot3d
    from workloads import WORKLOADS

    w = WORKLOADS[args.workload]
    faces = w.faces()
    br = w.br(faces)
    dev = torch.device("cuda:0")
    print(f"[bench] {w.describe()} N={w.n} tol={w.tol} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    solver = Solver(*faces, device=0)
    d_br = torch.from_numpy(br).to(dev)
    d_phi = torch.empty((w.nr, w.nt, w.np), dtype=torch.float64, device=dev)
    maxit = 500_000

    if args.profile_kernels:
        solver.solve_device(d_br, d_phi, 0.0, 8)
        ms_p, ms_r = solver.time_kernels(args.kernel_reps)
        # counter calibration: a device copy of N doubles whose source is not in
        # the 256 MB memory-side cache (a 1 GB fill runs in between)
        src = torch.ones(w.n, dtype=torch.float64, device=dev)
        flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        flush.fill_(2.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del flush
        print(json.dumps({"profile_kernels": w.describe(), "update_p_ms": ms_p, "update_r_ms": ms_r,
                          "copy_bytes_each_way": 8 * w.n, "launch": solver.stats()}), flush=True)
        solver.close()
        return

    for q in range(args.warmup):
        st, it, rr = solver.solve_device(d_br, d_phi, w.tol, maxit)
        print(f"[bench] warmup {q}: status={st} iters={it} true_relres={rr:.3e}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_iters = 0
    loop_ms = 0.0
    statuses = []
    for q in range(args.steps):
        st, it, rr = solver.solve_device(d_br, d_phi, w.tol, maxit)
        s = solver.stats()
        total_iters += it
        loop_ms += s["loop_ms"]
        statuses.append(st)
        print(f"[bench] step {q}: iters={it} solve_ms={s['solve_ms']:.1f} true_relres={rr:.3e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = solver.stats()
    phi_norm = float(torch.linalg.vector_norm(d_phi).item())

    it_per_s = total_iters / elapsed
    bytes_iter = 64.0 * w.n
    # per-kernel average launch time on the context stream (hipEvents)
    ms_p, ms_r = solver.time_kernels(args.kernel_reps)
    kern = {
        "update_p": {"alg_bytes_per_launch": 24.0 * w.n, "ms": ms_p},
        "update_r": {"alg_bytes_per_launch": 40.0 * w.n, "ms": ms_r},
    }
    for k, v in kern.items():
        v["gbs"] = v["alg_bytes_per_launch"] / (v["ms"] * 1e-3) / 1e9
    dom = max(kern, key=lambda k: kern[k]["ms"])
    traffic = load_traffic(w.name, dom)
    roofline = {"bound": "hbm", "achieved": round(kern[dom]["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kern[dom]["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_name(stats, dom),
                "alg_bytes_per_launch": kern[dom]["alg_bytes_per_launch"], "ms_per_launch": kern[dom]["ms"]}

    result = {
        "metric": "PCG iters/s + HBM GB/s (% peak) at 151x301x601; FP32-refined vs FP64 solve s",
        "value": round(it_per_s, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.describe(), "n": w.n, "tol": w.tol,
                   "br": f"dipole 5 + {w.nbip} power-law bipoles, seed {w.seed}",
                   "iters_per_solve": total_iters // max(1, args.steps), "parallelism": "1 GPU"},
        "roofline": roofline,
        "hbm_gbs_alg_per_iteration": round(it_per_s * bytes_iter / 1e9, 1),
        "hbm_frac_per_iteration": round(it_per_s * bytes_iter / 1e9 / HBM_PEAK_GBS, 4),
        "fp64_solve_s": round(elapsed / args.steps, 4),
        "kernels": {k: {"ms": round(v["ms"], 4), "gbs_alg": round(v["gbs"], 1)} for k, v in kern.items()},
        "loop_us_per_iter": round(loop_ms * 1e3 / max(1, total_iters), 2),
        "launch": {k: stats[k] for k in ("tile_p", "tile_r", "chunk_p", "chunk_r", "blocks_p", "blocks_r", "pitch")},
        "status": [pot3d.STATUS_NAMES.get(s, s) for s in statuses],
        "relres_true": stats["relres_true"],
        "phi_l2": phi_norm,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, faces, br, args.cpu_budget)
    solver.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
