#!/usr/bin/env python3
"""Throughput of LMMSE-CG equalisation of Zak-OTFS frames on one MI355X.

One step = one fused CG-LMMSE solve (Algorithm 1 with the relative-residual stop) of the
whole batch of the named workload, every iteration applying H and H^H on the fly, with
hard decisions.  The headline workload is the largest one-GPU batch: 128 frames of
(M, N) = (1024, 256), P = 16, 64-QAM, 30 dB, complex64 with the FP64 true-residual
refresh every 10 iterations.

The received frames y = H x + w are made by the FP64 oracle (complex128, rounded once to
complex64) in worker processes before this process touches the GPU; the GPU solves
exactly those y, inputs resident in HBM before the timed region.  The oracle's CG on a
spread sample of the frames is the cpu_baseline leg (timed on this host's cores) and the
reference for the line's NMSE and decision checks.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import hashlib
import json
import math
import multiprocessing
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "equalized OTFS symbols/sec (CG-LMMSE) @NMSE≤1e-5; p99 frame latency"
PEAK_HBM_GBS = 8000.0
NMSE_TARGET = 1e-5
DECISION_FP32_SLACK = 2.0 ** -20   # rounding allowance of an FP32 decision (signal units)
KERNEL_SRC = os.path.join(ROOT, "paper_2604_02266_amd", "csrc", "kernels.hip")
MAX_WORKERS = 16          # the CPU share of one GPU on the benchmark hosts
# FP64 refresh period per workload (the 128 x (1024, 256) configuration asks for 10)
REFRESH = {"batch128_1024x256": 10}
SECONDARY = "batch64_512x128"
SWEEP_RATES = (2000, 5000, 10000, 20000, 30000, 40000, 50000)

# Algorithmic bytes per element (complex64 vectors, 8 B per element; hard decisions 1 B),
# counted on the three-phase schedule of Algorithm 1:
#   init    b = H^H y -> c, p, x = 0              read y (8)            write c, p, x (24)
#   per iteration
#     P1: x += alpha p, p' = c + beta p, t = H p'  read x, c, p (24)     write x, p', t (24)
#     P2: a = H^H t + lam p'                      read t, p' (16)       write a (8)
#     P3: c -= alpha a                            read c, a (16)        write c (8)
#   finish  x += alpha p, decisions               read x, p (16)        write x (8), sym (1)
#   refresh (every k iterations) c = H^H (y - H x) - lam x: 40 B per element
# Gathered re-reads of a vector inside a pass, index tables and coefficients are not
# counted.
BYTES_INIT, BYTES_ITER, BYTES_FINISH, BYTES_REFRESH = 32.0, 96.0, 25.0, 40.0


def kernel_source_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# ----------------------------------------------------------------------------------------
# CPU side: the oracle in worker processes (forked before this process touches the GPU)
# ----------------------------------------------------------------------------------------
def _worker_init():
    # one BLAS thread per worker process (the library was loaded before the fork, so the
    # environment variables alone would come too late): the workers already fill the cores
    for v in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
        os.environ[v] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _job_received(frame):
    import oracle as O
    _, _, y = O.received_frame(frame)
    return y


def _job_solve(args):
    """The oracle as it stands: its operator and its FP64 CG on the given y, timed."""
    import oracle as O
    frame, y = args
    sp = frame.spec
    t0 = time.perf_counter()
    op = O.TwistedConvChannel(sp.M, sp.N, sp.h, sp.tau, sp.nu)
    x, it, rel = O.cg_lmmse(y, op, sp.lam, sp.max_iters, sp.tol)
    return x, it, rel, time.perf_counter() - t0


def spread(n, k):
    """k indices spread evenly over range(n)."""
    k = min(k, n)
    return sorted({int(round(i * (n - 1) / max(k - 1, 1))) for i in range(k)})


def cpu_phase(pool, workers, frames, sample, timed):
    """Oracle-made y for every frame, then the oracle's CG on the sample frames (the
    cpu_baseline leg when timed)."""
    ys = pool.map(_job_received, frames, chunksize=1)
    t0 = time.perf_counter()
    res = pool.map(_job_solve, [(frames[i], ys[i]) for i in sample], chunksize=1)
    wall = time.perf_counter() - t0
    refs = {i: r for i, r in zip(sample, res)}
    cpu = None
    if timed:
        syms = sum(frames[i].spec.E for i in sample)
        per = [r[3] for r in res]
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        cpu = {"value": syms / wall, "unit": "symbols/s", "cores": workers, "kind": "oracle",
               "host_cpus": cores,
               "single_worker_value": frames[sample[0]].spec.E / (sum(per) / len(per)),
               "sample": f"{len(sample)} of {len(frames)} frames spread over the batch (their "
                         f"own operator and FP64 NumPy CG with the same stop rule, on the same "
                         f"y as the GPU), one frame per worker process, {workers} workers on "
                         f"{cores} host CPUs: {wall:.1f} s wall, {sum(per):.1f} s CPU; "
                         f"single_worker_value = symbols per frame / mean CPU s per frame"}
    return ys, refs, cpu


# ----------------------------------------------------------------------------------------
# GPU side
# ----------------------------------------------------------------------------------------
def iters_refreshes(it, k, max_iters):
    if k <= 0:
        return 0
    return int(min(it, max_iters - 1) // k)


def launch_bytes(specs, iters, refresh):
    import numpy as np
    tot = 0.0
    for sp, it in zip(specs, iters):
        nref = iters_refreshes(int(it), refresh, sp.max_iters)
        tot += sp.E * (BYTES_INIT + BYTES_ITER * float(it) + BYTES_FINISH + BYTES_REFRESH * nref)
    return float(tot)


def check_against_oracle(O, np, frames, offs, x, sym, refs):
    """Worst NMSE over the sample frames, and the decisions that differ from the oracle's:
    all of them, and those not explained by the estimates (the oracle's estimate farther
    from a boundary than the GPU's estimate is from it).  None without oracle results."""
    if not refs:
        return None
    worst, diff, unexplained, n = 0.0, 0, 0, 0
    for i, r in refs.items():
        sp = frames[i].spec
        xg = x[offs[i]:offs[i + 1]]
        sg = sym[offs[i]:offs[i + 1]]
        worst = max(worst, O.nmse(xg, r[0]))
        # both decisions in the kernel's precision (the FP32 rule)
        ref_sym = O.qam_decide(r[0].astype(np.complex64), sp.qam, np.float32)
        d = np.nonzero(sg != ref_sym)[0]
        diff += int(d.size)
        if d.size:
            margin = O.decision_margin(r[0][d], sp.qam)
            err = np.abs(xg[d].astype(np.complex128) - r[0][d])
            unexplained += int(np.count_nonzero(margin >= err + DECISION_FP32_SLACK))
        n += sp.E
    return {"frames": len(refs), "nmse_worst": worst, "nmse_ok": bool(worst <= NMSE_TARGET),
            "decisions_compared": n, "decisions_differing": diff,
            "decisions_differing_unexplained": unexplained}


def time_solves(plan, y, xhat, dec, stats, steps, warmup, torch):
    for _ in range(warmup):
        plan.lmmse_cg(y, xhat, dec, stats)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.lmmse_cg(y, xhat, dec, stats)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_times(otfs, specs, y, xhat, dec, stats, reps, refresh, torch):
    """Fused-kernel durations from HIP events on the launch stream, and host-side time of
    each whole solve (launch to completion)."""
    sp0 = specs[0]
    tplan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol, refresh_every=refresh,
                      flags=otfs.TIME_KERNEL)
    kms, solve_ms = [], []
    for i in range(reps + 1):
        t1 = time.perf_counter()
        tplan.lmmse_cg(y, xhat, dec, stats)
        k = tplan.kernel_ms()
        if i > 0:
            kms.append(k)
            solve_ms.append((time.perf_counter() - t1) * 1e3)
    del tplan
    return kms, solve_ms


def copy_bandwidth(torch, nbytes=2 << 30, reps=5):
    """Device-to-device copy of nbytes with torch: read + write bytes / median time."""
    import numpy as np
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / float(np.median(ts)) / 1e9


def solve_block(otfs, O, np, torch, name, frames, ys, refs, steps, warmup, refresh, plain,
                copy_gbs):
    """Time the fused solve of one workload and check it against the oracle's sample."""
    specs = [f.spec for f in frames]
    sp0 = specs[0]
    offs = otfs.frame_offsets(specs)
    dev = torch.device("cuda")
    plan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol, refresh_every=refresh)
    E = plan.total_elems
    y = torch.from_numpy(np.concatenate(ys).astype(np.complex64)).to(dev)
    xhat = torch.empty_like(y)
    dec = torch.empty(E, dtype=torch.uint8, device=dev)
    stats = plan.new_stats()
    torch.cuda.synchronize()
    wall = time_solves(plan, y, xhat, dec, stats, steps, warmup, torch)
    value = E * steps / wall
    st = otfs.stats_numpy(stats)
    iters = st["iters"].astype(np.float64)
    xh = xhat.cpu().numpy()
    dh = dec.cpu().numpy()
    sym_tx = np.concatenate([f.sym for f in frames]).astype(np.int64)
    ser = float(np.mean(dh.astype(np.int64) != sym_tx))
    parity = check_against_oracle(O, np, frames, offs, xh, dh, refs)
    lb = launch_bytes(specs, iters, refresh)
    lds = bool(plan.tuned and plan.tuned.get("lds_gather"))
    kname = "k_cg_fused<0, 5> (LDS-windowed paired gathers)" if lds else "k_cg_fused"
    kms, solve_ms = kernel_times(otfs, specs, y, xhat, dec, stats, steps, refresh, torch)
    kavg = float(np.mean(kms))
    achieved = lb / (kavg * 1e-3) / 1e9
    out = {
        "value": value, "ms_per_step": wall * 1e3 / steps,
        "config": {"workload": name, "frames": len(specs), "M": sp0.M, "N": sp0.N, "P": sp0.P,
                   "qam": sp0.qam, "snr_db": sp0.snr_db, "max_iters": sp0.max_iters,
                   "rel_tol": sp0.tol, "refresh_every": refresh, "precision": "complex64"},
        "latency_ms": {"batch_p50": float(np.percentile(solve_ms, 50)),
                       "batch_p99": float(np.percentile(solve_ms, 99)),
                       "note": "whole-batch solve, every frame done by its end"},
        "iterations": {"mean": float(iters.mean()), "min": int(iters.min()),
                       "max": int(iters.max()),
                       "converged_frames": int(np.sum(st["status"] == otfs.FRAME_CONVERGED))},
        "ser_vs_transmitted": ser,
        "parity_vs_oracle": parity,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": load_traffic(name, refresh),
                     "kernel": (kname[:-1] + ", FP64 refresh inside the launch)" if lds and refresh
                                else kname + (" + k_refresh_u + k_refresh_c" if refresh else "")),
                     "kernel_ms": kavg,
                     "algorithmic_bytes_per_launch": lb,
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
    }
    if plain:
        out["plain_form"] = plain_block(otfs, O, np, torch, frames, ys, refs, refresh, offs)
    del plan, y, xhat, dec, stats
    torch.cuda.empty_cache()
    return out


def plain_block(otfs, O, np, torch, frames, ys, refs, refresh, offs, reps=3):
    """The plain form (one frame at a time, four unfused launches per iteration) on the
    same y, with a tiling made for one frame at a time; one warm-up, median of reps."""
    specs = [f.spec for f in frames]
    sp0 = specs[0]
    tile = max(512, max(sp.E for sp in specs) // 256)
    plan = otfs.Plan(specs, max_iters=sp0.max_iters, rel_tol=sp0.tol, tile_elems=tile)
    y = torch.from_numpy(np.concatenate(ys).astype(np.complex64)).to("cuda")
    xhat = torch.empty_like(y)
    dec = torch.empty(plan.total_elems, dtype=torch.uint8, device="cuda")
    stats = plan.new_stats()
    plan.lmmse_cg_plain(y, xhat, dec, stats)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t1 = time.perf_counter()
        plan.lmmse_cg_plain(y, xhat, dec, stats)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    tp = float(np.median(ts))
    parity = check_against_oracle(O, np, frames, offs, xhat.cpu().numpy(), dec.cpu().numpy(), refs)
    del plan, y, xhat, dec, stats
    return {"value": plan_elems(specs) / tp, "unit": "symbols/s", "ms_per_step": tp * 1e3,
            "runs": reps, "tile_elems": tile,
            "nmse_worst": None if parity is None else parity["nmse_worst"],
            "note": "no FP64 refresh in the plain form" if refresh else ""}


PEAK_MFMA_FP32_TFLOPS = 157.3


def dzt_block(otfs, np, torch, M, N, nframes, reps=10):
    """The front end's DZT (Eq. zak as the batched GEMM of Eq. zak_gemm on FP32 MFMA) of a
    batch of time-domain frames: 8 M N^2 real flops per frame, timed with HIP events."""
    x = torch.randn(nframes * M * N, dtype=torch.complex64, device="cuda")
    out = torch.empty_like(x)
    otfs.dzt(x, M, N, out=out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        otfs.dzt(x, M, N, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    flops = 8.0 * M * N * N * nframes
    del x, out
    return {"workload": f"{nframes} x ({M},{N}) time-domain frames", "ms": ms,
            "frames_per_s": nframes / (ms * 1e-3),
            "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12,
                         "peak": PEAK_MFMA_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / (ms * 1e-3) / 1e12 / PEAK_MFMA_FP32_TFLOPS,
                         "kernel": "k_dzt (v_mfma_f32_16x16x4_f32)"}}


def plan_elems(specs):
    return float(sum(sp.E for sp in specs))


def load_traffic(workload, refresh):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha() or int(t.get("refresh_every", 0)) != refresh:
        return None
    return t.get("traffic_bytes_per_launch")


# ----------------------------------------------------------------------------------------
# serving: Poisson arrival sweep
# ----------------------------------------------------------------------------------------
def serving_sweep(otfs, np, torch, frames, ys, rates, nframes, pool_bytes, step_iters=5,
                  seed=1004):
    """Poisson arrival streams of `nframes` frames (the workload's frames, cycled) at each
    offered rate: achieved offered rate, completed symbols/s and p50 / p99 / p99.9 latency
    from submit to completion (the server's clock).  A submitter thread paces the arrivals;
    the main thread polls the results (batched calls) into reused buffers, so host memory
    stays bounded and neither side waits on the other.  Latency runs from a frame's
    scheduled arrival (the server's clock from its submit, plus the generator's delay)."""
    import threading
    from collections import deque
    specs = [f.spec for f in frames]
    sp0 = specs[0]
    rng = np.random.default_rng(seed)
    out = []
    sw = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    try:
        with otfs.Server(pool_bytes, max_iters=sp0.max_iters, rel_tol=sp0.tol,
                         step_iters=step_iters) as srv:
            prep = [srv.prepare(sp) for sp in specs]
            bufs = [(np.empty(sp.E, dtype=np.complex64), np.empty(sp.E, dtype=np.uint8))
                    for sp in specs]
            for _ in range(2):   # warm-up: the host buffer pools and the kernels
                warm = [srv.submit(pp, yy) for pp, yy in zip(prep, ys)]
                for tk, pp, bb in zip(warm, prep, bufs):
                    srv.wait(tk, pp, timeout=120.0, out=bb)
            for ri, rate in enumerate(rates):
                arrivals = np.cumsum(rng.exponential(1.0 / rate, nframes))
                arrivals -= arrivals[0]
                shared = deque()
                t_sub = [None]
                t0 = time.perf_counter()

                def submitter():
                    # frames whose arrival time has passed go in one call; a frame's wait
                    # from its arrival to that call is added to its latency
                    n = 0
                    while n < nframes:
                        now = time.perf_counter() - t0
                        due = int(np.searchsorted(arrivals, now, side="right"))
                        if due <= n:
                            time.sleep(min(arrivals[n] - now, 2e-3))
                            continue
                        due = min(due, n + 256)
                        ks = [m % len(specs) for m in range(n, due)]
                        tks = srv.submit_many([prep[k] for k in ks], [ys[k] for k in ks])
                        shared.extend((tk, k, now - arrivals[m])
                                      for tk, k, m in zip(tks, ks, range(n, due)))
                        n = due
                    t_sub[0] = time.perf_counter() - t0

                th = threading.Thread(target=submitter)
                th.start()
                lat, syms, got = [], 0, 0
                mine = []
                while got < nframes:
                    while shared:
                        mine.append(shared.popleft())
                    if not mine:
                        time.sleep(5e-5)
                        continue
                    head = mine[:512]
                    res = srv.poll_many([h[0] for h in head], [bufs[h[1]] for h in head])
                    left = []
                    for h, r in zip(head, res):
                        if r is None:
                            left.append(h)
                            continue
                        lat.append(r[1] + h[2])
                        syms += specs[h[1]].E
                        got += 1
                    mine = left + mine[512:]
                    if len(left) == len(head):
                        time.sleep(5e-5)
                wall = time.perf_counter() - t0
                th.join()
                lat = np.array(lat) * 1e3
                out.append({"offered_frames_per_s": rate,
                            "achieved_offered_frames_per_s": nframes / t_sub[0] if t_sub[0] else None,
                            "completed_frames_per_s": nframes / wall,
                            "value": syms / wall, "unit": "symbols/s",
                            "latency_ms_p50": float(np.percentile(lat, 50)),
                            "latency_ms_p99": float(np.percentile(lat, 99)),
                            "latency_ms_p999": float(np.percentile(lat, 99.9))})
                print(f"[serving] {json.dumps(out[-1])}", file=sys.stderr, flush=True)
            st = srv.stats()
    finally:
        sys.setswitchinterval(sw)
    # the knee: the highest offered rate whose completed rate keeps up (within 5 %) with the
    # rate the load generator actually offered, and which the generator itself reached
    # (within 10 % of the nominal rate)
    knee = None
    for p in out:
        ach = p["achieved_offered_frames_per_s"] or 0.0
        if (p["completed_frames_per_s"] >= 0.95 * ach
                and ach >= 0.9 * p["offered_frames_per_s"]):
            knee = p
    return {"workload": "serving_uneven", "frames_per_point": nframes, "step_iters": step_iters,
            "pool_bytes": pool_bytes, "pool_bytes_peak": int(st.pool_bytes_peak),
            "points": out,
            "knee": None if knee is None else {"offered_frames_per_s": knee["offered_frames_per_s"],
                                               "value": knee["value"],
                                               "latency_ms_p99": knee["latency_ms_p99"]},
            "scheduler_ms": {"admit": st.ns_admit / 1e6, "step": st.ns_step / 1e6,
                             "gpu": st.ns_gpu / 1e6, "fetch": st.ns_fetch / 1e6},
            "note": "host buffers in and out (submit copies y, poll copies x_hat); Poisson "
                    "arrivals, frames of the uneven-batch shapes cycled"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch128_1024x256")
    ap.add_argument("--refresh", type=int, default=None,
                    help="FP64 refresh period (default: the workload's own, else none)")
    ap.add_argument("--cpu-frames", type=int, default=MAX_WORKERS,
                    help="oracle sample size (frames spread over the batch)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle: y made on the GPU (apply_H + noise), no parity line")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 64 x (512,128) block")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep")
    ap.add_argument("--sweep-rates", default=",".join(str(r) for r in SWEEP_RATES))
    ap.add_argument("--sweep-frames", type=int, default=5000)
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

    import workloads as W

    refresh = REFRESH.get(args.workload, 0) if args.refresh is None else args.refresh
    frames = list(W.iter_frames(args.workload))
    blocks = [(args.workload, frames, refresh)]
    if not args.no_secondary and args.workload != SECONDARY:
        blocks.append((SECONDARY, list(W.iter_frames(SECONDARY)), REFRESH.get(SECONDARY, 0)))
    serve_frames = None if args.no_serving else list(W.iter_frames("serving_uneven"))

    # ---- CPU phase: oracle-made inputs and the oracle's solves, before the GPU is touched ----
    cpu = None
    data = {}
    serve_ys = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        workers = max(1, min(cores or 1, MAX_WORKERS))
        print(f"[bench] oracle phase: {workers} workers", file=sys.stderr, flush=True)
        with multiprocessing.get_context("fork").Pool(workers, initializer=_worker_init) as pool:
            for bi, (name, frs, _) in enumerate(blocks):
                sample = spread(len(frs), args.cpu_frames)
                ys, refs, c = cpu_phase(pool, workers, frs, sample, timed=(bi == 0))
                data[name] = (ys, refs)
                if bi == 0:
                    cpu = c
                print(f"[bench] oracle phase done for {name}", file=sys.stderr, flush=True)
            if serve_frames is not None:
                serve_ys = pool.map(_job_received, serve_frames, chunksize=4)

    import torch

    import oracle as O
    import paper_2604_02266_amd as otfs

    if args.no_cpu:   # inputs made on the GPU: the library's H applied to the symbols + noise
        for name, frs, _ in blocks:
            data[name] = (gpu_made_y(otfs, np, torch, frs), {})
        if serve_frames is not None:
            serve_ys = gpu_made_y(otfs, np, torch, serve_frames)

    if args.calibrate_copy > 0:
        n = args.calibrate_copy // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    copy_gbs = copy_bandwidth(torch)
    results = []
    for bi, (name, frs, rf) in enumerate(blocks):
        ys, refs = data[name]
        print(f"[bench] gpu block {name}", file=sys.stderr, flush=True)
        results.append(solve_block(otfs, O, np, torch, name, frs, ys, refs, args.steps,
                                   args.warmup, rf, plain=(bi == 0 and not args.no_plain),
                                   copy_gbs=copy_gbs))

    main_res = results[0]
    par = main_res["parity_vs_oracle"]
    if par is not None and not par["nmse_ok"]:
        print(f"[bench] WARNING: NMSE {par['nmse_worst']:.3e} exceeds {NMSE_TARGET}",
              file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64",
        "data": "synthetic",
        "config": main_res["config"],
    }
    for k in ("latency_ms", "iterations", "ser_vs_transmitted", "parity_vs_oracle", "roofline",
              "plain_form"):
        if k in main_res:
            out[k] = main_res[k]
    if len(results) > 1:
        sec = results[1]
        out["secondary"] = {k: sec[k] for k in ("value", "ms_per_step", "config", "iterations",
                                                 "parity_vs_oracle", "roofline")}
    sp0 = frames[0].spec
    out["front_end_dzt"] = dzt_block(otfs, np, torch, sp0.M, sp0.N, len(frames))
    if serve_frames is not None:
        rates = [float(r) for r in args.sweep_rates.split(",") if r]
        out["serving"] = serving_sweep(otfs, np, torch, serve_frames, serve_ys, rates,
                                       args.sweep_frames, args.sweep_pool_gib << 30)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    out["build"] = otfs.build_info()   # the library's source stamp, checked against this tree
    print(json.dumps(out), flush=True)


def gpu_made_y(otfs, np, torch, frames):
    """y = H x + w with the library's H (for runs without the oracle, e.g. under a
    profiler): QAM points from the generator's symbol indices, the generator's noise."""
    specs = [f.spec for f in frames]
    plan = otfs.Plan(specs, max_iters=1, rel_tol=0.0)
    offs = otfs.frame_offsets(specs)
    x = np.empty(plan.total_elems, dtype=np.complex64)
    for i, f in enumerate(frames):
        m = int(round(math.sqrt(f.spec.qam)))
        s = math.sqrt(2.0 * (f.spec.qam - 1) / 3.0)
        ii, qq = np.divmod(np.asarray(f.sym, dtype=np.int64), m)
        x[offs[i]:offs[i + 1]] = ((2 * ii - (m - 1)) + 1j * (2 * qq - (m - 1))) / s
    y = plan.apply_H(torch.from_numpy(x).to("cuda")).cpu().numpy()
    y = y + np.concatenate([f.noise for f in frames]).astype(np.complex64)
    del plan
    return [y[offs[i]:offs[i + 1]] for i in range(len(frames))]


if __name__ == "__main__":
    main()
