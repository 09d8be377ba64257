#!/usr/bin/env python3
"""Throughput of LMMSE-CG equalisation of Zak-OTFS frames on one MI355X.

One step = one fused CG-LMMSE solve (Algorithm 1 with the relative-residual stop) of the
whole batch of the named workload, every iteration applying H and H^H on the fly, with
hard decisions.  Inputs (the received frames y) are synthesised on the GPU before the
timed region: QAM symbols from the seeded generator, y = H x + w with the library's own
otfs_apply_H and the generator's noise.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "equalized OTFS symbols/sec (CG-LMMSE) @NMSE≤1e-5; p99 frame latency"
PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2604_02266_amd", "csrc", "kernels.hip")

# Algorithmic bytes per element (complex64 vectors, 8 B per element; hard decisions 1 B),
# counted on the three-phase schedule of Algorithm 1 with the direction formed where the
# H product reads it (what the benchmark batch runs):
#   init    b = H^H y -> c, p, x = 0              read y (8)            write c, p, x (24)
#   per iteration
#     P1: x += alpha p, p' = c + beta p, t = H p'  read x, c, p (24)     write x, p', t (24)
#     P2: a = H^H t + lam p'                      read t, p' (16)       write a (8)
#     P3: c -= alpha a                            read c, a (16)        write c (8)
#   finish  x += alpha p, decisions               read x, p (16)        write x (8), sym (1)
# Gathered re-reads of a vector inside a pass, index tables and coefficients are not
# counted.  (Batches with more than 8 paths per frame form p' in a pass of its own, which
# moves 8 B more per element and iteration; those bytes are not counted either.)
BYTES_INIT, BYTES_ITER, BYTES_FINISH = 32.0, 96.0, 25.0


def kernel_source_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def qam_points_torch(torch, sym, Q):
    m = int(round(math.sqrt(Q)))
    s = math.sqrt(2.0 * (Q - 1) / 3.0)
    i_i = torch.div(sym, m, rounding_mode="floor")
    i_q = sym - i_i * m
    re = (2 * i_i - (m - 1)).to(torch.float32) / s
    im = (2 * i_q - (m - 1)).to(torch.float32) / s
    return torch.complex(re, im)


def _cpu_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    import oracle as O
    frame = args
    op, x, y = O.received_frame(frame)
    t0 = time.perf_counter()
    O.cg_lmmse(y, op, frame.spec.lam, frame.spec.max_iters, frame.spec.tol)
    return time.perf_counter() - t0, frame.spec.E


def _warm(_):
    import oracle  # noqa: F401
    return 0


def cpu_baseline(frames, nsample):
    """The FP64 oracle on a bounded sample of the workload's frames, one frame per worker
    process, wall clock over the whole sample (y synthesis excluded)."""
    from concurrent.futures import ProcessPoolExecutor
    sample = frames[:nsample]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(cores, len(sample), 16))
    import multiprocessing
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("fork")) as ex:
        list(ex.map(_warm, range(workers)))                  # imports outside the timing
        t0 = time.perf_counter()
        res = list(ex.map(_cpu_worker, sample))
        wall = time.perf_counter() - t0
    syms = sum(e for _, e in res)
    return {"value": syms / wall, "unit": "symbols/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(sample)} of {len(frames)} frames, FP64 NumPy CG with the same stop "
                      f"rule, {workers} processes, {wall:.1f} s wall, "
                      f"{sum(t for t, _ in res):.1f} s CPU"}


def load_traffic(workload, launch_bytes):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t.get("traffic_bytes_per_launch")


def serving_leg(otfs, W, workload, torch, step_iters=5, seed=1004):
    """Frames of `workload` offered to the server: first all at once (throughput), then as
    a Poisson stream at half that rate (latency from submit to completion)."""
    import numpy as np
    frames = list(W.iter_frames(workload))
    specs = [f.spec for f in frames]
    sp0 = specs[0]
    # received frames, synthesised on the GPU and handed to the server as host buffers
    plan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol)
    offs = otfs.frame_offsets(specs)
    dev = torch.device("cuda")
    sym = torch.from_numpy(np.concatenate([f.sym for f in frames])).to(dev)
    x = torch.empty(plan.total_elems, dtype=torch.complex64, device=dev)
    for i, f in enumerate(frames):
        x[offs[i]:offs[i + 1]] = qam_points_torch(torch, sym[offs[i]:offs[i + 1]], f.spec.qam)
    noise = torch.from_numpy(np.concatenate([f.noise for f in frames]).astype(np.complex64))
    y = (plan.apply_H(x).cpu() + noise).numpy()
    del plan, x, sym
    ys = [y[offs[i]:offs[i + 1]] for i in range(len(specs))]
    total = float(offs[-1])

    def run(srv, arrivals):
        t0 = time.perf_counter()
        tickets = []
        for i, (sp, yy) in enumerate(zip(specs, ys)):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(sp, yy))
        lat = [srv.wait(t, sp, timeout=120.0)[3] for t, sp in zip(tickets, specs)]
        return time.perf_counter() - t0, np.array(lat) * 1e3

    pool = 8 << 30
    with otfs.Server(pool, max_iters=sp0.max_iters, rel_tol=sp0.tol,
                     step_iters=step_iters) as srv:
        run(srv, np.zeros(len(specs)))                       # warm-up
        wall, lat_burst = run(srv, np.zeros(len(specs)))
        rate = len(specs) / wall
        gaps = np.random.default_rng(seed).exponential(2.0 / rate, len(specs))
        wall_p, lat_p = run(srv, np.cumsum(gaps) - gaps[0])
        st = srv.stats()
    return {"workload": workload, "frames": len(specs), "step_iters": step_iters,
            "pool_bytes": pool, "pool_bytes_peak": int(st.pool_bytes_peak),
            "burst": {"value": total / wall, "unit": "symbols/s", "frames_per_s": rate,
                      "latency_ms_p50": float(np.percentile(lat_burst, 50)),
                      "latency_ms_p99": float(np.percentile(lat_burst, 99))},
            "poisson_half_rate": {"offered_frames_per_s": rate / 2,
                                  "value": total / wall_p, "unit": "symbols/s",
                                  "latency_ms_p50": float(np.percentile(lat_p, 50)),
                                  "latency_ms_p99": float(np.percentile(lat_p, 99))},
            "note": "host buffers in and out (submit copies y, poll copies x_hat)"}


def serving_sweep(otfs, W, workload, torch, rates, nframes, pool_bytes, step_iters=5,
                  seed=1004):
    """Poisson arrival streams of `nframes` frames (the workload's frames, cycled) at each
    offered rate: achieved offered rate, completed symbols/s and p50 / p99 / p99.9 latency
    from submit to completion.  Results are polled while frames are being submitted, so
    host memory stays bounded."""
    import numpy as np
    from collections import deque
    frames = list(W.iter_frames(workload))
    specs = [f.spec for f in frames]
    sp0 = specs[0]
    plan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol)
    offs = otfs.frame_offsets(specs)
    dev = torch.device("cuda")
    sym = torch.from_numpy(np.concatenate([f.sym for f in frames])).to(dev)
    x = torch.empty(plan.total_elems, dtype=torch.complex64, device=dev)
    for i, f in enumerate(frames):
        x[offs[i]:offs[i + 1]] = qam_points_torch(torch, sym[offs[i]:offs[i + 1]], f.spec.qam)
    noise = torch.from_numpy(np.concatenate([f.noise for f in frames]).astype(np.complex64))
    y = (plan.apply_H(x).cpu() + noise).numpy()
    del plan, x, sym
    ys = [y[offs[i]:offs[i + 1]] for i in range(len(specs))]
    rng = np.random.default_rng(seed)
    out = []
    with otfs.Server(pool_bytes, max_iters=sp0.max_iters, rel_tol=sp0.tol,
                     step_iters=step_iters) as srv:
        warm = [srv.submit(sp, yy) for sp, yy in zip(specs, ys)]      # warm-up
        for tk, sp in zip(warm, specs):
            srv.wait(tk, sp, timeout=120.0)
        for rate in rates:
            arrivals = np.cumsum(rng.exponential(1.0 / rate, nframes))
            arrivals -= arrivals[0]
            pending, lat, syms = deque(), [], 0
            t0 = time.perf_counter()
            for n in range(nframes):
                k = n % len(specs)
                wait = arrivals[n] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                pending.append((srv.submit(specs[k], ys[k]), k))
                while pending:
                    r = srv.poll(pending[0][0], specs[pending[0][1]])
                    if r is None:
                        break
                    lat.append(r[3])
                    syms += specs[pending[0][1]].E
                    pending.popleft()
            t_sub = time.perf_counter() - t0
            for tk, k in pending:
                r = srv.wait(tk, specs[k], timeout=300.0)
                lat.append(r[3])
                syms += specs[k].E
            wall = time.perf_counter() - t0
            lat = np.array(lat) * 1e3
            out.append({"offered_frames_per_s": rate,
                        "achieved_offered_frames_per_s": nframes / t_sub if t_sub > 0 else None,
                        "completed_frames_per_s": nframes / wall,
                        "value": syms / wall, "unit": "symbols/s",
                        "latency_ms_p50": float(np.percentile(lat, 50)),
                        "latency_ms_p99": float(np.percentile(lat, 99)),
                        "latency_ms_p999": float(np.percentile(lat, 99.9))})
            print(json.dumps(out[-1]), file=sys.stderr, flush=True)
    return {"workload": workload, "frames_per_point": nframes, "step_iters": step_iters,
            "pool_bytes": pool_bytes, "points": out,
            "note": "host buffers in and out (submit copies y, poll copies x_hat)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64_512x128")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-frames", type=int, default=6)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop leg")
    ap.add_argument("--serving-workload", default="serving_uneven")
    ap.add_argument("--serving-sweep", default="", metavar="RATES",
                    help="instead of the benchmark, sweep the serving loop over Poisson "
                         "arrival rates (comma-separated frames/s) and print that JSON line")
    ap.add_argument("--sweep-frames", type=int, default=10000)
    ap.add_argument("--sweep-pool-gib", type=int, default=64)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="also run one plain device-to-device copy of BYTES bytes (reference "
                         "for hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: frames are independent, so the path shards by "
              "splitting the frame list across GPUs with no exchange; only "
              "the one-GPU figure is measured.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2604_02266_amd as otfs
    import workloads as W

    if args.serving_sweep:
        rates = [float(r) for r in args.serving_sweep.split(",") if r]
        res = serving_sweep(otfs, W, args.serving_workload, torch, rates, args.sweep_frames,
                            args.sweep_pool_gib << 30)
        print(json.dumps({"serving_sweep": res}))
        return

    frames = list(W.iter_frames(args.workload))
    specs = [f.spec for f in frames]
    sp0 = specs[0]
    # the CPU leg runs first, before this process touches the GPU (its workers are forked)
    cpu = None if args.no_cpu else cpu_baseline(frames, args.cpu_frames)

    plan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol)
    E = plan.total_elems
    dev = torch.device("cuda")

    # inputs, resident before timing
    sym = torch.from_numpy(np.concatenate([f.sym for f in frames])).to(dev)
    x = torch.empty(E, dtype=torch.complex64, device=dev)
    offs = otfs.frame_offsets(specs)
    for i, f in enumerate(frames):
        x[offs[i]:offs[i + 1]] = qam_points_torch(torch, sym[offs[i]:offs[i + 1]], f.spec.qam)
    noise = torch.from_numpy(np.concatenate([f.noise for f in frames]).astype(np.complex64)).to(dev)
    y = plan.apply_H(x)
    y += noise
    xhat = torch.empty_like(y)
    dec = torch.empty(E, dtype=torch.uint8, device=dev)
    stats = plan.new_stats()
    torch.cuda.synchronize()

    if args.calibrate_copy > 0:
        n = args.calibrate_copy // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        plan.lmmse_cg(y, xhat, dec, stats)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.lmmse_cg(y, xhat, dec, stats)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = E * args.steps / wall

    st = otfs.stats_numpy(stats)
    iters = st["iters"].astype(np.float64)
    sizes = np.diff(offs).astype(np.float64)
    launch_bytes = float(np.sum(sizes * (BYTES_INIT + BYTES_ITER * iters + BYTES_FINISH)))
    ser = float(np.mean(dec.cpu().numpy() != sym.cpu().numpy().astype(np.uint8)))

    # fused-kernel duration from HIP events on the launch stream, and per-solve latency
    tplan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol, flags=otfs.TIME_KERNEL)
    kms, solve_ms = [], []
    for i in range(args.steps + 1):
        t1 = time.perf_counter()
        tplan.lmmse_cg(y, xhat, dec, stats)
        k = tplan.kernel_ms()
        if i > 0:
            kms.append(k)
            solve_ms.append((time.perf_counter() - t1) * 1e3)
    kavg = float(np.mean(kms))
    achieved = launch_bytes / (kavg * 1e-3) / 1e9
    del tplan

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64",
        "data": "synthetic",
        "config": {"workload": args.workload, "frames": len(specs), "M": sp0.M, "N": sp0.N,
                   "P": sp0.P, "qam": sp0.qam, "snr_db": sp0.snr_db,
                   "max_iters": sp0.max_iters, "rel_tol": sp0.tol},
        "latency_ms": {"batch_p50": float(np.percentile(solve_ms, 50)),
                       "batch_p99": float(np.percentile(solve_ms, 99)),
                       "note": "whole-batch solve, every frame done by its end"},
        "iterations": {"mean": float(iters.mean()), "min": int(iters.min()),
                       "max": int(iters.max()),
                       "converged_frames": int(np.sum(st["status"] == otfs.FRAME_CONVERGED))},
        "ser_vs_transmitted": ser,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": load_traffic(args.workload, launch_bytes),
                     "kernel": "k_cg_fused", "kernel_ms": kavg,
                     "algorithmic_bytes_per_launch": launch_bytes},
    }

    if not args.no_plain:
        t1 = time.perf_counter()
        plan.lmmse_cg_plain(y, xhat, dec, stats)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t1
        out["plain_form"] = {"value": E / tp, "unit": "symbols/s", "ms_per_step": tp * 1e3}

    if not args.no_serving:
        del plan, y, xhat, dec, stats, x, noise, sym
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(otfs, W, args.serving_workload, torch)

    if cpu is not None:
        out["cpu_baseline"] = cpu

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
