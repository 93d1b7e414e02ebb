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


# algorithmic bytes per unknown of each iteration kernel, and the kernel-name
# fragments that identify it in a trace
# fragments that identify it in a trace.  One-sweep form: the even sweeps
# leave x to the odd ones (32 N: read r, p_old; write r, p), the odd sweeps
# update x for both (48 N: also read and write x); "sweep" is the sweep that
# updates x every time (POT3D_SWEEP_X=1).
KERNEL_KEYS = {"sweep_even": (32.0, ("stencil_sweep<", "double, 1>")),
               "sweep_odd": (48.0, ("stencil_sweep<", "double, 2>")),
               "sweep": (48.0, ("stencil_sweep<", "double, 0>")),
               "update_p": (24.0, (", 2, double>",)), "update_r": (40.0, (", 3, double>",)),
               # the r/x update of the two-pass and phi-line iterations, x once per pair
               "update_r_skip": (24.0, (", 4, double>",)), "update_r_pair": (48.0, (", 5, double>",)),
               "sweep_fp32_even": (16.0, ("stencil_sweep<", "float, 1>")),
               "sweep_fp32_odd": (24.0, ("stencil_sweep<", "float, 2>")),
               "line": (16.0, ("line_solve_kernel<",))}


def summarize_pmc(workload: str, fetch_dir: str, write_dir: str):
    """HBM bytes per launch of the iteration kernels from FETCH_SIZE and
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
    for key, (per_unknown, frags) in KERNEL_KEYS.items():
        names = [k for k in fetch if all(f in k for f in frags)]
        if not names:
            continue
        name = names[0]
        # dispatches that ran (the graph's launches after convergence return at once)
        real_f = [x for x in fetch[name] if x > 0.1 * max(fetch[name])]
        real_w = [x for x in write[name] if x > 0.1 * max(write[name])]
        fb = statistics.median(real_f) * f_scale
        wb = statistics.median(real_w) * w_scale
        alg = per_unknown * n
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
    xm = {"sweep": 0, "sweep_even": 1, "sweep_odd": 2}
    if which in xm:
        return f"stencil_sweep<{stats['sweep_rows']},double,{xm[which]}>"
    tile = stats["tile_p"] if which == "update_p" else stats["tile_r"]
    mode = "2" if which == "update_p" else "4|5"   # the r/x update alternates its two pairing modes
    if tile > 100:
        return f"stencil_wave<{tile - 100},{mode},double>"
    return f"stencil_march<{tile},{mode},double>"


def host_cpu():
    """The host's CPU model and core counts (from /proc/cpuinfo and the affinity mask)."""
    model, logical, cores, cur = None, 0, set(), None
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                continue
            key, val = (t.strip() for t in line.split(":", 1))
            if key == "processor":
                logical += 1
            elif key == "model name" and model is None:
                model = val
            elif key == "physical id":
                cur = val
            elif key == "core id":
                cores.add((cur, val))
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": logical or os.cpu_count(), "physical_cores": len(cores) or None,
            "usable_cpus": usable}


def cpu_baseline(w, faces, br, budget_s: float):
    """The oracle's fixed-count iterations on the host cores: all threads
    OpenMP gives it (the value), then one thread (the paper's serial baseline,
    Sec. 4.1) on a shorter sample."""
    import oracle

    rf, tf, pf = faces
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br)

    def timed(budget):
        # a warm-up run, two short runs to size the sample (per-iteration time
        # and the per-call setup), then a run of about `budget` seconds
        oracle.pcg(coef, b, 0.0, 1)
        t0 = time.perf_counter()
        oracle.pcg(coef, b, 0.0, 2)
        t2 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.pcg(coef, b, 0.0, 6)
        t6 = time.perf_counter() - t0
        per = max(1e-4, (t6 - t2) / 4)
        setup = max(0.0, t2 - 2 * per)
        k = max(3, int((budget - setup) / per))
        t0 = time.perf_counter()
        _, iters, _, _ = oracle.pcg(coef, b, 0.0, k)
        return iters, time.perf_counter() - t0

    threads = oracle.set_threads(0)
    iters, dt = timed(budget_s)
    oracle.set_threads(1)
    iters1, dt1 = timed(budget_s / 2)
    oracle.set_threads(threads)
    return {"value": iters / dt, "unit": "iter/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} FP64 Jacobi-PCG iterations of {w.describe()} (tol=0, fixed count), "
                      f"{dt:.1f} s, OpenMP threads={threads}; assembly excluded",
            "one_thread": {"value": iters1 / dt1, "unit": "iter/s", "cores": 1,
                           "sample": f"{iters1} iterations, {dt1:.1f} s, OpenMP threads=1"},
            "host": host_cpu()}


def rocm_version():
    try:
        return open("/opt/rocm/.info/version").read().strip()
    except OSError:
        return None


def stream_ceiling(torch, dev, n):
    """Practical HBM ceilings of plain streaming kernels on vectors of n
    doubles: a copy (1 read + 1 write) and addcmul (3 reads + 1 write),
    timed with events on the current stream."""
    a = torch.rand(n, dtype=torch.float64, device=dev)
    b, c, d = torch.rand_like(a), torch.rand_like(a), torch.empty_like(a)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_copy = timed(lambda: d.copy_(a))
    t_acm = timed(lambda: torch.addcmul(a, b, c, out=d))
    out = {"vector_bytes": 8 * n, "copy_gbs": round(16.0 * n / t_copy / 1e9, 1),
           "addcmul_3r1w_gbs": round(32.0 * n / t_acm / 1e9, 1)}
    del a, b, c, d
    return out


def golden_samples(name):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def err_vs_samples(torch, d_phi, g):
    """Max |Phi - Phi_oracle| / max |Phi_oracle| at the golden file's sampled indices."""
    if not g or "phi" not in g:
        return None
    import numpy as np

    idx = torch.tensor(g["indices"], dtype=torch.long, device=d_phi.device)
    got = d_phi.reshape(-1)[idx].cpu().numpy()
    return float(np.abs(got - np.array(g["phi"])).max() / g["phi_max_abs"])


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def fifo_latencies(arrivals, service):
    """Latencies of a single FIFO server that runs one request at a time."""
    free, out = 0.0, []
    for a, s in zip(arrivals, service):
        start = max(a, free)
        free = start + s
        out.append(free - a)
    return out


def serve_trace(server, reqs, arrivals, log):
    """Submit each request at its arrival time (host clock, relative to the
    first step) and step the server until all are done.  Returns per-request
    (latency s, iters, status, relres_true) and the makespan."""
    k = len(reqs)
    ids = [None] * k
    done = [None] * k
    nxt = 0
    t0 = time.perf_counter()
    t_sub = [0.0] * k
    while any(d is None for d in done):
        now = time.perf_counter() - t0
        while nxt < k and arrivals[nxt] <= now:
            w, faces, br = reqs[nxt]
            ids[nxt] = server.submit(*faces, br, w.tol, 1_000_000)
            t_sub[nxt] = server.info(ids[nxt])["t_submit"]
            nxt += 1
        active, queued, _ = server.step()
        for q in range(nxt):
            if done[q] is None:
                info = server.info(ids[q])
                if info["done"]:
                    server.take(ids[q])
                    done[q] = (info["t_done"] - t_sub[q], info["iters"], info["status"], info["relres_true"])
                    log(f"[serve]   request {q} {info['nr']}x{info['nt']}x{info['np']} done: "
                        f"latency {done[q][0]:.3f} s, iters {info['iters']}")
        if active == 0 and queued == 0 and nxt < k:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    return done, time.perf_counter() - t0


def serve_saturation(reqs, precision, slots, log, cache_budget=None):
    """The same requests through back-to-back single solves (cached contexts,
    host arrays, as the server takes them) and through the server with every
    request queued at once.  Returns solves/s, latencies and whether every
    served solve took the same iterations as alone."""
    import numpy as np

    from paper_1709_01126_amd import Server, Solver

    solvers, service, seq = {}, [], []
    for w, faces, br in reqs:
        key = (w.nr, w.nt, w.np)
        if key not in solvers:
            solvers[key] = Solver(*faces, precision=precision)
            solvers[key].solve(br, w.tol, 1_000_000)   # warm-up
    for w, faces, br in reqs:
        t = time.perf_counter()
        _, st, it, rr = solvers[(w.nr, w.nt, w.np)].solve(br, w.tol, 1_000_000)
        service.append(time.perf_counter() - t)
        seq.append(it)
    for sv in solvers.values():
        sv.close()
    k = len(reqs)
    seq_lat = fifo_latencies([0.0] * k, service)
    with Server(precision=precision, max_slots=slots) as server:
        if cache_budget is not None:
            server.set_cache_budget(cache_budget)
        warm = []
        for key in sorted({(w.nr, w.nt, w.np) for w, _, _ in reqs}):
            warm.append(next(r for r in reqs if (r[0].nr, r[0].nt, r[0].np) == key))
        serve_trace(server, warm, [0.0] * len(warm), lambda m: None)
        res, span = serve_trace(server, reqs, [0.0] * k, lambda m: None)
    lat = [r[0] for r in res]
    out = {"requests": k, "sequential_solves_per_s": round(k / sum(service), 4),
           "server_solves_per_s": round(k / span, 4),
           "server_over_sequential": round(sum(service) / span, 3),
           "server_p50_s": round(percentile(lat, 50), 4), "server_p99_s": round(percentile(lat, 99), 4),
           "sequential_p50_s": round(percentile(seq_lat, 50), 4), "sequential_p99_s": round(percentile(seq_lat, 99), 4),
           "iters_equal_alone": all(r[1] == s_ for r, s_ in zip(res, seq)),
           "all_ok": all(r[2] == 0 for r in res), "max_relres_true": max(r[3] for r in res)}
    log(f"[serve] {json.dumps(out)}")
    return out


def serve_leg(n_requests, slots, log):
    """Bounded serving measurement for the default line: the first
    n_requests of the mixed-size trace, all queued at once, FP64 and
    FP32-refined."""
    from paper_1709_01126_amd import FP32_REFINED, FP64
    from workloads import configs

    reqs = []
    for q in range(n_requests):
        w = configs.serve_request(q)
        faces = w.faces()
        reqs.append((w, faces, w.br(faces)))
    sizes = {}
    for w, _, _ in reqs:
        sizes[f"{w.nr}x{w.nt}x{w.np}"] = sizes.get(f"{w.nr}x{w.nt}x{w.np}", 0) + 1
    out = {"trace": f"first {n_requests} requests of the serving trace (sizes uniform over "
                    f"{['x'.join(map(str, z)) for z in configs.SERVE_SIZES]}, 50..500 bipoles, tol 1e-9), "
                    f"all queued at once", "sizes": sizes, "slots": slots}
    for name, prec in (("fp64", FP64), ("fp32_refined", FP32_REFINED)):
        log(f"[serve] {name}: {n_requests} requests at saturation")
        out[name] = serve_saturation(reqs, prec, slots, log)
    return out


def serve_main(args):
    """Continuous-batching serving on the mixed-size request trace."""
    import numpy as np
    import torch  # noqa: F401  (initialises the device the way the tests do)

    from paper_1709_01126_amd import FP32_REFINED, FP64, Server, Solver
    from workloads import configs

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    k = args.serve_requests
    reqs = []
    for q in range(k):
        w = configs.serve_request(q)
        faces = w.faces()
        reqs.append((w, faces, w.br(faces)))
    sizes = sorted({(w.nr, w.nt, w.np) for w, _, _ in reqs})
    log(f"[serve] {k} requests, sizes {sizes}, {args.serve_slots} slots")
    arrivals_cfg = configs.poisson_arrivals(k, args.serve_rate, seed=17)
    result = {"metric": "serving: solves/s and p50/p99 latency, continuous batching vs sequential solves",
              "unit": "solves/s", "n_gpus": 1, "data": "synthetic", "higher_is_better": True,
              "config": {"workload": f"serve trace of {k} requests: sizes uniform over {list(configs.SERVE_SIZES)}, "
                                     f"50..500 bipoles, tol 1e-9", "slots": args.serve_slots,
                         "rate_per_s": args.serve_rate,
                         "cache_budget_bytes": args.serve_cache_budget if args.serve_cache_budget is not None
                         else 256 * 2 ** 20},
              "modes": {}}
    for name, prec in (("fp64", FP64), ("fp32_refined", FP32_REFINED)):
        # sequential: one solve at a time through pot3d_solve, contexts cached per grid
        solvers = {}
        for w, faces, br in reqs:
            key = (w.nr, w.nt, w.np)
            if key not in solvers:
                solvers[key] = Solver(*faces, precision=prec)
                solvers[key].solve(br, w.tol, 1_000_000)   # warm-up
        service, seq_res = [], []
        for q, (w, faces, br) in enumerate(reqs):
            t = time.perf_counter()
            _, st, it, rr = solvers[(w.nr, w.nt, w.np)].solve(br, w.tol, 1_000_000)
            service.append(time.perf_counter() - t)
            seq_res.append((it, st, rr))
        for sv in solvers.values():
            sv.close()
        seq_rate = k / sum(service)
        log(f"[serve] {name} sequential: {seq_rate:.3f} solves/s, mean solve {np.mean(service):.3f} s")
        mode = {"sequential": {"solves_per_s": round(seq_rate, 4), "mean_solve_s": round(float(np.mean(service)), 4),
                               "max_relres_true": max(r[2] for r in seq_res)}}
        with Server(precision=prec, max_slots=args.serve_slots) as server:
            if args.serve_cache_budget is not None:
                server.set_cache_budget(args.serve_cache_budget)
            # warm-up: one request per size, so each grid has a cached context
            warm = []
            for key in sizes:
                w, faces, br = next(r for r in reqs if (r[0].nr, r[0].nt, r[0].np) == key)
                warm.append((w, faces, br))
            serve_trace(server, warm, [0.0] * len(warm), lambda m: None)
            runs = [("saturation", [0.0] * k), (f"poisson_{args.serve_rate:g}", list(arrivals_cfg))]
            for label, arr in runs:
                log(f"[serve] {name} server, arrivals: {label}")
                res, span = serve_trace(server, reqs, arr, log)
                lat = [r[0] for r in res]
                seq_lat = fifo_latencies(arr, service)
                mode[label] = {
                    "server": {"solves_per_s": round(k / span, 4), "p50_s": round(percentile(lat, 50), 4),
                               "p99_s": round(percentile(lat, 99), 4),
                               "max_relres_true": max(r[3] for r in res),
                               "status_ok": sum(r[2] == 0 for r in res)},
                    "sequential_fifo": {"p50_s": round(percentile(seq_lat, 50), 4),
                                        "p99_s": round(percentile(seq_lat, 99), 4)},
                    "iters_equal_sequential": all(r[1] == s[0] for r, s in zip(res, seq_res)),
                }
                log(f"[serve] {name} {label}: {json.dumps(mode[label])}")
            # a sustainable rate: 70% of the measured server throughput
            lam = 0.7 * mode["saturation"]["server"]["solves_per_s"]
            arr = list(configs.poisson_arrivals(k, lam, seed=19))
            log(f"[serve] {name} server, arrivals: poisson at {lam:.3f}/s (70% of saturation)")
            res, span = serve_trace(server, reqs, arr, log)
            lat = [r[0] for r in res]
            seq_lat = fifo_latencies(arr, service)
            mode["poisson_sustainable"] = {
                "rate_per_s": round(lam, 4),
                "server": {"p50_s": round(percentile(lat, 50), 4), "p99_s": round(percentile(lat, 99), 4)},
                "sequential_fifo": {"p50_s": round(percentile(seq_lat, 50), 4),
                                    "p99_s": round(percentile(seq_lat, 99), 4)},
            }
            mode["server_stats"] = server.stats()
        result["modes"][name] = mode
    # one size at a time, 8 requests each, all queued at once: where batching
    # pays (small, cache-resident, latency-bound solves) and where it cannot
    # (bandwidth-bound ones)
    result["per_size"] = {}
    for size in configs.SERVE_SIZES:
        reqs_s = []
        for q in range(8):
            wq = configs.Workload(f"size_{size}_{q}", *size, 1e-9, 300 + q, "ratio3", "bipoles", nbip=100)
            faces = wq.faces()
            reqs_s.append((wq, faces, wq.br(faces)))
        key = "x".join(map(str, size))
        result["per_size"][key] = {name: serve_saturation(reqs_s, prec, args.serve_slots, log)
                                   for name, prec in (("fp64", FP64), ("fp32_refined", FP32_REFINED))}
    result["value"] = result["modes"]["fp64"]["saturation"]["server"]["solves_per_s"]
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bipole_151x301x601")
    ap.add_argument("--kernel-reps", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders (FETCH_SIZE, WRITE_SIZE) of a --profile-kernels "
                         "run into profiles/traffic_<workload>.json and exit")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="short run for hardware counters: a few iterations and --kernel-reps timed launches of "
                         "the FP64 sweep and the two passes, a few phi-line iterations, the FP32 sweep, and one "
                         "device copy of N doubles (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="continuous-batching serving benchmark on the mixed-size request trace (own JSON line)")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-cache-budget", type=float, default=None,
                    help="bytes streamed per iteration by the batch (server default: 256 MiB; 0 = no limit)")
    ap.add_argument("--no-closed-wall", action="store_true", help="skip the closed-wall solve")
    ap.add_argument("--no-refined", action="store_true", help="skip the FP32-refined solves of the default run")
    ap.add_argument("--no-line", action="store_true", help="skip the phi-line preconditioner solves")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the streaming-ceiling measurement")
    ap.add_argument("--no-large", action="store_true", help="skip the fixed-count run on the large grid")
    ap.add_argument("--large-workload", default="bipole_301x641x1281")
    ap.add_argument("--serve-leg", type=int, default=12,
                    help="requests of the bounded serving measurement in the default line (0: skip)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.workload, *args.summarize_pmc)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this solver runs on a single device (asked for --gpus {args.gpus}); "
              "a decomposition over several GPUs (radial slabs with a halo exchange per sweep) is not built.",
              file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_main(args)
        return

    import numpy as np
    import torch

    from paper_1709_01126_amd import FP32_REFINED, Solver, pot3d
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
        # both iteration forms: the one-sweep kernel, then the two passes
        solver.solve_device(d_br, d_phi, 0.0, 8)
        ms_se, ms_so = solver.time_kernels(args.kernel_reps)
        solver.set_iteration(pot3d.ITER_TWO_PASS)
        solver.solve_device(d_br, d_phi, 0.0, 8)
        ms_p, ms_r = solver.time_kernels(args.kernel_reps)
        solver.set_iteration(pot3d.ITER_ONE_SWEEP)
        # the phi-line preconditioner's passes, and the FP32 sweep of the refined mode
        solver.set_preconditioner(pot3d.PC_PHI_LINE)
        solver.solve_device(d_br, d_phi, 0.0, 8)
        solver.set_preconditioner(pot3d.PC_JACOBI)
        with Solver(*faces, precision=FP32_REFINED, device=0) as s32:
            s32.solve_device(d_br, d_phi, 0.0, 8)
            ms_s32e, ms_s32o = s32.time_kernels(args.kernel_reps)
            fp32_form = "one-sweep" if s32.stats()["iteration"] == pot3d.ITER_ONE_SWEEP else "two-pass"
        # counter calibration: a device copy of N doubles whose source is not in
        # the 256 MB memory-side cache (a 1 GB fill runs in between)
        src = torch.ones(w.n, dtype=torch.float64, device=dev)
        flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        flush.fill_(2.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del flush
        print(json.dumps({"profile_kernels": w.describe(), "sweep_even_ms": ms_se, "sweep_odd_ms": ms_so,
                          "update_p_ms": ms_p, "update_r_ms": ms_r,
                          "fp32_inner": {"form": fp32_form, "ms": [ms_s32e, ms_s32o],
                                         "kernels": "even, odd sweep" if fp32_form == "one-sweep" else
                                                    "p update, r/x update"},
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

    # the field B = -grad Phi of the solution on the cell faces (reads Phi,
    # writes three face arrays: about 32 bytes per unknown); before the kernel
    # timing, which overwrites the solution
    nr_, nt_, np_ = w.nr, w.nt, w.np
    fbr = torch.empty((nr_ + 1, nt_, np_), dtype=torch.float64, device=dev)
    fbt = torch.empty((nr_, nt_ + 1, np_), dtype=torch.float64, device=dev)
    fbp = torch.empty((nr_, nt_, np_), dtype=torch.float64, device=dev)
    sptr = torch.cuda.current_stream(dev).cuda_stream
    pot3d.pot3d_field_device(solver.ctx, fbr.data_ptr(), fbt.data_ptr(), fbp.data_ptr(), sptr)
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        rcf = pot3d.pot3d_field_device(solver.ctx, fbr.data_ptr(), fbt.data_ptr(), fbp.data_ptr(), sptr)
    tf_ = (time.perf_counter() - t0) / reps
    field = {"ms": round(tf_ * 1e3, 3), "status": pot3d.STATUS_NAMES.get(rcf, rcf),
             "gbs_alg": round((8.0 * w.n + 8.0 * (fbr.numel() + fbt.numel() + fbp.numel())) / tf_ / 1e9, 1)}
    del fbr, fbt, fbp
    it_per_s = total_iters / elapsed
    one_sweep = stats["iteration"] == pot3d.ITER_ONE_SWEEP
    bytes_iter = stats["bytes_per_iter"]
    # per-kernel average launch time as the kernels run in a solve
    # (device wall-clock stamps per launch inside a replayed graph)
    ms_a, ms_b = solver.time_kernels(args.kernel_reps)
    paired = one_sweep and abs(bytes_iter - 40.0 * w.n) < 0.5
    if paired:
        kern = {"sweep_even": {"alg_bytes_per_launch": KERNEL_KEYS["sweep_even"][0] * w.n, "ms": ms_a},
                "sweep_odd": {"alg_bytes_per_launch": KERNEL_KEYS["sweep_odd"][0] * w.n, "ms": ms_b}}
    elif one_sweep:
        kern = {"sweep": {"alg_bytes_per_launch": KERNEL_KEYS["sweep"][0] * w.n, "ms": 0.5 * (ms_a + ms_b)}}
    else:
        kern = {
            "update_p": {"alg_bytes_per_launch": KERNEL_KEYS["update_p"][0] * w.n, "ms": ms_a},
            # the r/x update's mean over a pair of iterations (x once per pair: 24 N and 48 N)
            "update_r": {"alg_bytes_per_launch": (bytes_iter / w.n - KERNEL_KEYS["update_p"][0]) * w.n, "ms": ms_b},
        }
    for k, v in kern.items():
        v["gbs"] = v["alg_bytes_per_launch"] / (v["ms"] * 1e-3) / 1e9
    if paired:
        # the sweeps run in pairs (even, odd) that alternate through the solve:
        # the pair is the unit, 80 N bytes over the two launch times, quoted per
        # launch (40 N over their mean)
        ev, od = kern["sweep_even"], kern["sweep_odd"]
        ms_mean = 0.5 * (ev["ms"] + od["ms"])
        gbs = 40.0 * w.n / (ms_mean * 1e-3) / 1e9
        t_ev, t_od = load_traffic(w.name, "sweep_even"), load_traffic(w.name, "sweep_odd")
        traffic = None if t_ev is None or t_od is None else 0.5 * (t_ev + t_od)
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": f"{kernel_name(stats, 'sweep_even')} + {kernel_name(stats, 'sweep_odd')}",
                    "alg_bytes_per_launch": 40.0 * w.n, "ms_per_launch": ms_mean,
                    "basis": "40 N bytes per launch, the mean of an even sweep (32 N: read r, p_old; write r, p) "
                             "and an odd one (48 N: also read and write x, for both sweeps)"}
    else:
        dom = max(kern, key=lambda k: kern[k]["ms"])
        ms_mean = kern[dom]["ms"]
        roofline = {"bound": "hbm", "achieved": round(kern[dom]["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(kern[dom]["gbs"] / HBM_PEAK_GBS, 4), "traffic": load_traffic(w.name, dom),
                    "kernel": kernel_name(stats, dom),
                    "alg_bytes_per_launch": kern[dom]["alg_bytes_per_launch"], "ms_per_launch": ms_mean,
                    "basis": f"{KERNEL_KEYS[dom][0]:g} N bytes per launch: what this kernel must move"}
    if one_sweep:
        # the same launch time on the textbook two-pass basis of one PCG
        # iteration (64 N: read r, p, x and re-read p, r; write p, x, r), which
        # is what an iteration costs without the one-sweep rearrangement, and
        # on the sweep that updates x every time (48 N)
        roofline["achieved_64N_basis"] = round(64.0 * w.n / (ms_mean * 1e-3) / 1e9, 1)
        roofline["frac_64N_basis"] = round(roofline["achieved_64N_basis"] / HBM_PEAK_GBS, 4)
        roofline["achieved_48N_basis"] = round(48.0 * w.n / (ms_mean * 1e-3) / 1e9, 1)
        roofline["frac_48N_basis"] = round(roofline["achieved_48N_basis"] / HBM_PEAK_GBS, 4)

    result = {
        "metric": "PCG iters/s + HBM GB/s (% peak) at 151x301x601; FP32-refined vs FP64 solve s",
        "value": round(it_per_s, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": None,   # one GPU: no scaling claim
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
        "iteration": "one-sweep" if one_sweep else "two-pass",
        "launch": ({k: stats[k] for k in ("sweep_rows", "chunk_s", "blocks_s", "pitch")} if one_sweep else
                   {k: stats[k] for k in ("tile_p", "tile_r", "chunk_p", "chunk_r", "blocks_p", "blocks_r", "pitch")}),
        "status": [pot3d.STATUS_NAMES.get(s, s) for s in statuses],
        "field": field,
        "relres_true": stats["relres_true"],
        "phi_l2": phi_norm,
        "max_rel_err_vs_oracle_samples": err_vs_samples(torch, d_phi, golden_samples(w.name)),
        "rocm": rocm_version(), "torch": torch.__version__,
    }
    if one_sweep:
        # the two-pass form of the same FP64 iteration, one solve, for comparison
        solver.set_iteration(pot3d.ITER_TWO_PASS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2, it2, rr2 = solver.solve_device(d_br, d_phi, w.tol, maxit)
        torch.cuda.synchronize()
        t2 = time.perf_counter() - t0
        result["two_pass"] = {"iters_per_s": round(it2 / t2, 2), "iters": it2, "solve_s": round(t2, 4),
                              "status": pot3d.STATUS_NAMES.get(st2, st2), "relres_true": rr2}
        print(f"[bench] two-pass: {it2 / t2:.1f} it/s ({it2} iters)", file=sys.stderr, flush=True)
        solver.set_iteration(pot3d.ITER_ONE_SWEEP)
    if not args.no_closed_wall:
        # the closed-wall upper boundary (Br = 0 on R1) on the same grid and data, one solve
        cw = Solver(*faces, upper_bc=pot3d.UPPER_CLOSED_WALL, device=0)
        d_phi_cw = torch.empty_like(d_phi)
        cw.solve_device(d_br, d_phi_cw, w.tol, maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st3, it3, rr3 = cw.solve_device(d_br, d_phi_cw, w.tol, maxit)
        torch.cuda.synchronize()
        t3 = time.perf_counter() - t0
        result["closed_wall"] = {"iters_per_s": round(it3 / t3, 2), "iters": it3, "solve_s": round(t3, 4),
                                 "status": pot3d.STATUS_NAMES.get(st3, st3), "relres_true": rr3}
        print(f"[bench] closed wall: {it3 / t3:.1f} it/s ({it3} iters)", file=sys.stderr, flush=True)
        cw.close()
        del d_phi_cw
    if not args.no_line:
        # the phi-line block preconditioner on the same grid and data: fewer
        # iterations, 76 N bytes each on average (direction update on z, r/x
        # update with x once per pair, line pass)
        solver.set_preconditioner(pot3d.PC_PHI_LINE)
        d_phi_l = torch.empty_like(d_phi)
        stl, itl, rrl = solver.solve_device(d_br, d_phi_l, w.tol, maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(max(1, args.steps)):
            stl, itl, rrl = solver.solve_device(d_br, d_phi_l, w.tol, maxit)
        torch.cuda.synchronize()
        tl = (time.perf_counter() - t0) / max(1, args.steps)
        sl = solver.stats()
        result["phi_line"] = {
            "solve_s": round(tl, 4), "speedup_vs_point_jacobi": round(result["fp64_solve_s"] / tl, 3),
            "iters": itl, "iters_point_jacobi": result["config"]["iters_per_solve"],
            "iters_per_s": round(itl / tl, 2), "loop_us_per_iter": round(sl["loop_ms"] * 1e3 / max(1, itl), 2),
            "bytes_per_unknown": round(sl["bytes_per_iter"] / w.n, 3),
            "gbs_alg": round(sl["bytes_per_iter"] * itl / (sl["loop_ms"] * 1e-3) / 1e9, 1),
            "status": pot3d.STATUS_NAMES.get(stl, stl), "relres_true": rrl,
            "max_rel_err_vs_oracle_samples": err_vs_samples(torch, d_phi_l, golden_samples(w.name + "_phi_line")),
            "max_rel_diff_vs_point_jacobi": float(torch.max(torch.abs(d_phi_l - d_phi)).item()
                                                  / torch.max(torch.abs(d_phi)).item())}
        print(f"[bench] phi-line: {tl:.3f} s/solve ({itl} iters)", file=sys.stderr, flush=True)
        solver.set_preconditioner(pot3d.PC_JACOBI)
        del d_phi_l
    if not args.no_refined:
        # FP32-refined solves of the same problem to the same FP64 residual
        phi64 = d_phi.clone()
        solver.close()
        solver = Solver(*faces, precision=FP32_REFINED, device=0)
        st, it, rr = solver.solve_device(d_br, d_phi, w.tol, maxit)
        print(f"[bench] refined warmup: status={st} inner iters={it} true_relres={rr:.3e}", file=sys.stderr,
              flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(args.steps):
            st, it, rr = solver.solve_device(d_br, d_phi, w.tol, maxit)
        torch.cuda.synchronize()
        t_ref = (time.perf_counter() - t0) / args.steps
        rs = solver.stats()
        diff = float(torch.max(torch.abs(d_phi - phi64)).item() / torch.max(torch.abs(phi64)).item())
        result["fp32_refined"] = {"solve_s": round(t_ref, 4), "speedup_vs_fp64": round(result["fp64_solve_s"] / t_ref, 3),
                                  "mode": "reliable updates (the FP32 direction continues across FP64 residual "
                                          "replacements), inner tol 0.1 (the library default for this mode)",
                                  "inner_iters": it, "outer": rs["outer"], "relres_true": rr,
                                  "status": pot3d.STATUS_NAMES.get(st, st),
                                  "max_rel_err_vs_oracle_samples": err_vs_samples(torch, d_phi,
                                                                                  golden_samples(w.name)),
                                  "max_rel_diff_vs_fp64_gpu": diff}
        print(f"[bench] refined: {t_ref:.3f} s/solve ({it} inner iters, {rs['outer']} outer)", file=sys.stderr,
              flush=True)
        # the mixed-precision configuration as first stated: plain defect
        # correction, each inner FP32 PCG restarted and run to 1e-5
        solver.set_refinement_mode(pot3d.REFINE_RESTART)
        solver.set_refinement(1e-5, 50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st5, it5, rr5 = solver.solve_device(d_br, d_phi, w.tol, maxit)
        torch.cuda.synchronize()
        t5 = time.perf_counter() - t0
        r5 = solver.stats()
        result["fp32_refined"]["restart_inner_1e-5"] = {
            "solve_s": round(t5, 4), "speedup_vs_fp64": round(result["fp64_solve_s"] / t5, 3), "inner_iters": it5,
            "outer": r5["outer"], "relres_true": rr5, "status": pot3d.STATUS_NAMES.get(st5, st5),
            "max_rel_err_vs_oracle_samples": err_vs_samples(torch, d_phi, golden_samples(w.name))}
        print(f"[bench] refined, restarts at inner tol 1e-5: {t5:.3f} s ({it5} inner iters, {r5['outer']} outer)",
              file=sys.stderr, flush=True)
        if not args.no_line:
            # both directions at once: FP32 inner iterations with the phi-line
            # preconditioner (reliable updates, the default inner tolerance)
            solver.set_refinement_mode(pot3d.REFINE_RELIABLE)
            solver.set_refinement(0.1, 50)
            solver.set_preconditioner(pot3d.PC_PHI_LINE)
            solver.solve_device(d_br, d_phi, w.tol, maxit)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for q in range(max(1, args.steps)):
                stl, itl, rrl = solver.solve_device(d_br, d_phi, w.tol, maxit)
            torch.cuda.synchronize()
            tl = (time.perf_counter() - t0) / max(1, args.steps)
            rl = solver.stats()
            result["fp32_refined"]["phi_line"] = {
                "solve_s": round(tl, 4), "speedup_vs_fp64": round(result["fp64_solve_s"] / tl, 3),
                "inner_iters": itl, "outer": rl["outer"], "relres_true": rrl,
                "status": pot3d.STATUS_NAMES.get(stl, stl),
                "max_rel_err_vs_oracle_samples": err_vs_samples(torch, d_phi, golden_samples(w.name + "_phi_line"))}
            print(f"[bench] refined with the phi-line preconditioner: {tl:.3f} s ({itl} inner iters, "
                  f"{rl['outer']} outer)", file=sys.stderr, flush=True)
    solver.close()
    del d_phi, d_br
    torch.cuda.empty_cache()
    if not args.no_ceiling:
        # practical ceilings of plain streaming kernels, at this workload's
        # vector size and at 2 GB per vector (nothing reused from the 256 MB
        # memory-side cache)
        result["stream_ceiling"] = [stream_ceiling(torch, dev, w.n), stream_ceiling(torch, dev, 1 << 28)]
        torch.cuda.empty_cache()
        print(f"[bench] streaming ceilings: {result['stream_ceiling']}", file=sys.stderr, flush=True)
    if not args.no_large:
        result["large_grid"] = large_grid_leg(torch, dev, args.large_workload)
        torch.cuda.empty_cache()
    if args.serve_leg > 0:
        result["serving"] = serve_leg(args.serve_leg, args.serve_slots,
                                      lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, faces, br, args.cpu_budget)
    print(json.dumps(result), flush=True)


def large_grid_leg(torch, dev, name):
    """One GPU's share at its full shape (default 301 x 641 x 1281, 247M
    unknowns, 2 GB per vector): a short fixed-count run (no stopping test
    reached), its per-iteration loop time and the sweep kernel's launch time.
    The surface data are the workload's dipole alone (5 cos theta): a
    fixed-count iteration does the same work whatever the values, and the
    2000-bipole map takes most of a minute to sample on the host."""
    from paper_1709_01126_amd import Solver
    from workloads import WORKLOADS, magnetograms

    w = WORKLOADS[name]
    faces = w.faces()
    br = magnetograms.br_dipole(faces[1], faces[2], 5.0)
    print(f"[bench] large grid {w.describe()}: N={w.n}", file=sys.stderr, flush=True)
    with Solver(*faces, device=0) as s:
        d_br = torch.from_numpy(br).to(dev)
        d_phi = torch.empty((w.nr, w.nt, w.np), dtype=torch.float64, device=dev)
        s.solve_device(d_br, d_phi, 0.0, 8)
        k = 40
        st, it, rr = s.solve_device(d_br, d_phi, 0.0, k)
        stats = s.stats()
        ms_e, ms_o = s.time_kernels(8)
        ms_sweep = 0.5 * (ms_e + ms_o)
        del d_phi, d_br
    loop_us = stats["loop_ms"] * 1e3 / max(1, it)
    out = {"workload": w.describe(), "data": "dipole 5 cos(theta)", "n": w.n, "fixed_iters": it, "loop_us_per_iter": round(loop_us, 2),
           "iters_per_s": round(1e6 / loop_us, 2),
           "gbs_alg_per_iteration": round(stats["bytes_per_iter"] / (loop_us * 1e-6) / 1e9, 1),
           "sweep_ms_even_odd": [round(ms_e, 4), round(ms_o, 4)], "sweep_ms_mean": round(ms_sweep, 4),
           "sweep_traffic_even_odd": [load_traffic(w.name, "sweep_even"), load_traffic(w.name, "sweep_odd")],
           "sweep_gbs_alg": round(stats["bytes_per_iter"] / (ms_sweep * 1e-3) / 1e9, 1),
           "sweep_frac": round(stats["bytes_per_iter"] / (ms_sweep * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "launch": {k2: stats[k2] for k2 in ("sweep_rows", "chunk_s", "blocks_s", "pitch")}}
    print(f"[bench] large grid: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
