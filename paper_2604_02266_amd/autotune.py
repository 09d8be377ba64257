"""Autotuner of the fused CG-LMMSE launch shape.

The fused solve has a few knobs that do not change what is computed, only how the work
is cut and scheduled: the tiling of frames into workgroup bands (elements per tile, which
sets how many workgroups cooperate on a frame and how many frames run at once on an
XCD), whether the H pass forms the direction p' = c + beta p inside its gathers or in a
pass of its own, and the LDS budget for staged gather windows.  The best setting depends
on the frame shapes, the path count, the batch size and the modes (refresh, stored table).

tune() searches these knobs for one batch on the current device: every candidate plan
solves the same received frames; its fused solve is timed with HIP events on the launch
stream (median of `reps` after a warm-up) and its estimate is checked against the default
plan's (NMSE <= 1e-6: a candidate changes the rounding order of the per-tile partial
sums, nothing else).  The winner and the whole search table are stored in tuned.json
beside this module, keyed by the batch signature (frame shapes, batch-size bucket, path
bucket, modes).  Plan applies a stored winner by default (lookup()), and the serving
loop takes per-shape tiles from the same file (serving_tiles()).

    python -m paper_2604_02266_amd.autotune --workload batch128_1024x256 --refresh 10
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_PATH = os.environ.get("OTFS_TUNED") or os.path.join(HERE, "tuned.json")

# the flag bits of the header that the tuner may set (the others are the caller's)
_SPLIT_DIRECTION = 1 << 6
_LDS_GATHER = 1 << 8
_D_STORED_BF16, _Y_BF16, _D_STORED_C64 = 1 << 0, 1 << 1, 1 << 7


def _pow2_ceil(n: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(n, 1)))))


def path_bucket(P: int) -> int:
    return 8 if P <= 8 else (16 if P <= 16 else 64)


def signature(frames: Sequence, refresh_every: int = 0, flags: int = 0) -> str:
    """Batch signature: the set of frame shapes, the batch size rounded up to a power of
    two, the largest path count's bucket, and the modes that change the kernels."""
    shapes = sorted({(int(f.M), int(f.N)) for f in frames})
    P = max(int(np.asarray(f.tau).shape[0]) for f in frames) if frames else 0
    sd = "c64" if flags & _D_STORED_C64 else ("bf16" if flags & _D_STORED_BF16 else "none")
    return ("+".join(f"{M}x{N}" for M, N in shapes) + f"|n{_pow2_ceil(len(frames))}"
            f"|p{path_bucket(P)}|r{int(refresh_every > 0)}|d{sd}|y{int(bool(flags & _Y_BF16))}")


def _load() -> Dict:
    if not os.path.exists(CACHE_PATH):
        return {"batches": {}, "serving": {}}
    with open(CACHE_PATH) as f:
        d = json.load(f)
    d.setdefault("batches", {})
    d.setdefault("serving", {})
    return d


def lookup(frames: Sequence, refresh_every: int = 0, flags: int = 0) -> Optional[Dict]:
    """The stored winner for this batch signature: {"tile_elems", "split_direction",
    "stage_bytes", "lds_gather"}, or None."""
    ent = _load()["batches"].get(signature(frames, refresh_every, flags))
    return None if ent is None else ent["best"]


def serving_tiles() -> Dict[str, int]:
    """Per-shape tile sizes for the serving loop: {"MxN": tile_elems}."""
    return {k: int(v["tile_elems"]) for k, v in _load()["serving"].items()}


def candidates(frames: Sequence, cus: int = 256) -> List[Dict]:
    """Tilings from the frame sizes and the machine (tiles per frame for the largest frame,
    and tiles per CU for the whole batch), crossed with the direction form and, for frames
    whose rows split into 16-byte pairs, the LDS-windowed gathers."""
    Emax = max(int(f.M) * int(f.N) for f in frames)
    Etot = sum(int(f.M) * int(f.N) for f in frames)
    Nmax = max(int(f.N) for f in frames)
    tiles = set()
    for t in (1, 2, 4, 8, 16):
        if t <= Nmax:
            tiles.add(int(math.ceil(Emax / t)))
    for w in (0.5, 1.0, 2.0):
        tiles.add(max(512, int(Etot / (cus * w))))
    tiles = sorted(t for t in tiles if t >= 512)
    pairs = any(int(f.M) % 128 == 0 for f in frames)
    out = []
    for te in tiles:
        out.append({"tile_elems": te, "split_direction": False, "stage_bytes": 0,
                    "lds_gather": False})
        if max(int(np.asarray(f.tau).shape[0]) for f in frames) <= 8:
            out.append({"tile_elems": te, "split_direction": True, "stage_bytes": 0,
                        "lds_gather": False})
        if pairs:
            out.append({"tile_elems": te, "split_direction": False, "stage_bytes": 0,
                        "lds_gather": True})
    return out


def _received(otfs, torch, frames, seed=7):
    """Received frames for timing: the library's own H applied to random QAM points plus
    noise at the frames' SNR (their values do not affect the timing of a capped solve)."""
    rng = np.random.default_rng(seed)
    plan = otfs.Plan(frames, max_iters=1, rel_tol=0.0, tune=False)
    x = np.empty(plan.total_elems, dtype=np.complex64)
    o = 0
    for f in frames:
        E = int(f.M) * int(f.N)
        Q = int(getattr(f, "qam", 0) or 4)
        m = int(round(math.sqrt(Q)))
        s = math.sqrt(2.0 * (Q - 1) / 3.0)
        ii = rng.integers(0, m, E)
        qq = rng.integers(0, m, E)
        x[o:o + E] = ((2 * ii - (m - 1)) + 1j * (2 * qq - (m - 1))) / s
        o += E
    y = plan.apply_H(torch.from_numpy(x).to("cuda"))
    lam = np.concatenate([np.full(int(f.M) * int(f.N), float(f.lam)) for f in frames])
    w = (rng.standard_normal(o) + 1j * rng.standard_normal(o)) * np.sqrt(lam / 2.0)
    y = y + torch.from_numpy(w.astype(np.complex64)).to("cuda")
    del plan
    return y


def _time(otfs, torch, frames, y, cand, max_iters, rel_tol, refresh_every, flags, reps):
    fl = flags | otfs.TIME_KERNEL | (_SPLIT_DIRECTION if cand["split_direction"] else 0)
    fl |= _LDS_GATHER if cand.get("lds_gather") else 0
    plan = otfs.Plan(frames, max_iters=max_iters, rel_tol=rel_tol, refresh_every=refresh_every,
                     flags=fl, tile_elems=cand["tile_elems"],
                     stage_bytes=cand["stage_bytes"], tune=False)
    xh = torch.empty_like(y)
    ks = []
    for r in range(reps + 1):
        plan.lmmse_cg(y, xh)
        k = plan.kernel_ms()
        if r:
            ks.append(k)
    info = plan.info()
    del plan
    return float(np.median(ks)), xh, int(info.grid)


def tune(frames: Sequence, max_iters: int = 50, rel_tol: float = 1e-6, refresh_every: int = 0,
         flags: int = 0, reps: int = 3, save: bool = True, log=print) -> Dict:
    """Search the candidates for this batch on the current device; store the winner."""
    import torch

    import paper_2604_02266_amd as otfs
    y = _received(otfs, torch, frames)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    table = []
    ref = None
    for cand in candidates(frames, cus):
        try:
            ms, xh, grid = _time(otfs, torch, frames, y, cand, max_iters, rel_tol,
                                 refresh_every, flags, reps)
        except Exception as e:          # a tiling that cannot run (too many tiles for a frame)
            table.append(dict(cand, ms=None, error=str(e)))
            continue
        x = xh.cpu().numpy()
        if ref is None:
            ref = x
        nm = float(np.vdot(x - ref, x - ref).real / max(np.vdot(ref, ref).real, 1e-300))
        row = dict(cand, ms=ms, grid=grid, nmse_vs_first=nm, ok=bool(nm <= 1e-6))
        table.append(row)
        log(f"[tune] {json.dumps(row)}")
    good = [r for r in table if r.get("ok")]
    if not good:
        raise RuntimeError("no candidate ran")
    best = min(good, key=lambda r: r["ms"])
    sig = signature(frames, refresh_every, flags)
    ent = {"best": {k: best.get(k, False) for k in ("tile_elems", "split_direction", "stage_bytes",
                                                     "lds_gather")},
           "ms": best["ms"], "device": torch.cuda.get_device_name(0),
           "date": time.strftime("%Y-%m-%d"), "table": table}
    if save:
        d = _load()
        d["batches"][sig] = ent
        with open(CACHE_PATH, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    return {"signature": sig, **ent}


def tune_serving_shapes(shapes, P=16, reps=3, save=True, log=print) -> Dict[str, int]:
    """Per-shape tile of the serving loop: a batch of one frame of each shape, solved alone
    (the latency of a lone frame is what the serving tile trades against the throughput of
    many), timed over tiles of 1..16 per frame; store {"MxN": tile_elems}."""
    import workloads as W
    out = {}
    rng = np.random.default_rng(1004)
    for (M, N) in shapes:
        fr = W.small_frame(rng, M, N, P, (0, max(1, M // 16)), (-max(1, N // 8), max(1, N // 8)),
                           qam=16, snr_db=20.0, max_iters=50, tol=1e-6)
        res = tune([fr.spec] * 8, save=False, reps=reps, log=log)
        out[f"{M}x{N}"] = {"tile_elems": int(res["best"]["tile_elems"]), "ms_8_frames": res["ms"]}
    if save:
        d = _load()
        d["serving"].update(out)
        with open(CACHE_PATH, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", action="append", required=True,
                    help="named workload (repeatable)")
    ap.add_argument("--refresh", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--serving-shapes", default="",
                    help="also tune serving tiles for these shapes, e.g. 128x32,256x64")
    args = ap.parse_args(argv)
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as W
    for name in args.workload:
        specs = W.make_frame_specs(name)
        mi, tol = specs[0].max_iters, specs[0].tol
        res = tune(specs, max_iters=mi, rel_tol=tol, refresh_every=args.refresh,
                   flags=args.flags, reps=args.reps)
        print(json.dumps({"workload": name, "signature": res["signature"], "best": res["best"],
                          "ms": res["ms"]}), flush=True)
    if args.serving_shapes:
        shapes = [tuple(int(v) for v in s.split("x")) for s in args.serving_shapes.split(",")]
        print(json.dumps({"serving": tune_serving_shapes(shapes, reps=args.reps)}), flush=True)


if __name__ == "__main__":
    main()
