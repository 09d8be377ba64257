"""BER-driven iteration budget (Sec. IV-C, "BER-driven iteration selection").

The paper fixes the CG iteration count offline: for every operating point (grid size,
modulation, SNR) it records the bit error rate after each iteration, finds the first
iteration at which the BER has converged by the relative-change rule of Eq.
ber_convergence (r_xi = (BER_{xi-1} - BER_xi) / max(BER_{xi-1}, zeta) < eta, xi >= 2), and
takes the largest such iteration over all points as the budget.

This module measures the BER curves on the device: for each point a batch of frames is
solved once with otfs_lmmse_cg_trace, which records the bit errors (Gray map per axis) of
every iteration's decisions; the received frames are made by the library's own channel
operator applied to random QAM symbols plus noise at the point's SNR.

    python -m paper_2604_02266_amd.ber_profile --shape 128x32 --qam 16 --snr 0,5,10,15,20,25,30
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
from typing import Dict, List, Sequence

import numpy as np

ETA, ZETA = 1e-2, 1e-12      # the values of Sec. IV-C


def convergence_iteration(ber: Sequence[float], eta: float = ETA, zeta: float = ZETA) -> int:
    """First iteration xi >= 2 (1-based) whose signed relative BER change is below eta;
    len(ber) when none is."""
    for xi in range(2, len(ber) + 1):
        prev, cur = float(ber[xi - 2]), float(ber[xi - 1])
        if (prev - cur) / max(prev, zeta) < eta:
            return xi
    return len(ber)


def ber_curve(otfs, torch, frames, max_iters: int, seed: int = 0) -> np.ndarray:
    """BER after each of max_iters CG iterations over a batch of frame specs (fixed count)."""
    rng = np.random.default_rng(seed)
    plan = otfs.Plan(frames, max_iters=max_iters, rel_tol=0.0, tune=False)
    E = plan.total_elems
    sym = np.empty(E, dtype=np.uint8)
    x = np.empty(E, dtype=np.complex64)
    lam = np.empty(E, dtype=np.float64)
    bits = 0
    o = 0
    for f in frames:
        n = int(f.M) * int(f.N)
        Q = int(f.qam)
        m = int(round(math.sqrt(Q)))
        s = math.sqrt(2.0 * (Q - 1) / 3.0)
        idx = rng.integers(0, Q, n)
        sym[o:o + n] = idx
        x[o:o + n] = ((2 * (idx // m) - (m - 1)) + 1j * (2 * (idx % m) - (m - 1))) / s
        lam[o:o + n] = float(f.lam)
        bits += n * 2 * int(round(math.log2(m)))
        o += n
    y = plan.apply_H(torch.from_numpy(x).to("cuda"))
    w = (rng.standard_normal(E) + 1j * rng.standard_normal(E)) * np.sqrt(lam / 2.0)
    y = y + torch.from_numpy(w.astype(np.complex64)).to("cuda")
    tx = torch.from_numpy(sym).to("cuda")
    _, _, errs = plan.lmmse_cg_trace(y, tx)
    return errs.sum(dim=1).cpu().numpy().astype(np.float64) / bits


def profile(points: List[Dict], max_iters: int = 30, frames_per_point: int = 8, seed: int = 1,
            log=print) -> Dict:
    """points: dicts with M, N, P, qam, snr_db (and optional delay/doppler spans).  Returns
    the per-point curves, convergence iterations and the budget (their maximum)."""
    import torch

    import paper_2604_02266_amd as otfs
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as W
    rng = np.random.default_rng(seed)
    out = []
    for pt in points:
        M, N, P = int(pt["M"]), int(pt["N"]), int(pt["P"])
        dt = int(pt.get("delay_span", max(1, M // 16)))
        dv = int(pt.get("doppler_span", max(1, N // 8)))
        frames = [W.small_frame(rng, M, N, P, (0, dt), (-dv, dv), qam=int(pt["qam"]),
                                snr_db=float(pt["snr_db"]), max_iters=max_iters, tol=0.0).spec
                  for _ in range(frames_per_point)]
        ber = ber_curve(otfs, torch, frames, max_iters, seed=int(rng.integers(1 << 30)))
        xi = convergence_iteration(ber)
        row = dict(pt, ber=[float(b) for b in ber], converged_at=xi, ber_at_convergence=float(ber[xi - 1]),
                   ber_min=float(ber.min()), ber_min_at=int(np.argmin(ber)) + 1)
        out.append(row)
        log(f"[ber] {M}x{N} P={P} {pt['qam']}-QAM {pt['snr_db']} dB: converged at {xi} "
            f"(BER {ber[xi - 1]:.3e}; lowest {ber.min():.3e} at {row['ber_min_at']})")
    return {"points": out, "budget": max(r["converged_at"] for r in out), "eta": ETA, "zeta": ZETA}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--shape", action="append", default=None, help="MxN (repeatable)")
    ap.add_argument("--paths", type=int, default=6)
    ap.add_argument("--qam", default="4,16")
    ap.add_argument("--snr", default="0,5,10,15,20,25,30")
    ap.add_argument("--max-iters", type=int, default=30)
    ap.add_argument("--frames", type=int, default=8)
    args = ap.parse_args(argv)
    shapes = [tuple(int(v) for v in s.split("x")) for s in (args.shape or ["128x32"])]
    points = [dict(M=M, N=N, P=args.paths, qam=int(q), snr_db=float(s))
              for (M, N) in shapes for q in args.qam.split(",") for s in args.snr.split(",")]
    res = profile(points, max_iters=args.max_iters, frames_per_point=args.frames)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
