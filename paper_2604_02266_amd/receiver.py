"""The Zak-OTFS receiver chain on the device (Sec. III-A pipeline, Fig. otfs_pipeline):

  received pilot and data frames (time domain)
    -> DZT of every frame (Eq. zak, the batched GEMM of Eq. zak_gemm on MFMA; otfs_dzt)
    -> the channel's dominant paths from the pilot (Eqs. heff_hadamard, heff_thres;
       otfs_plan_paths_from_pilot), without a host round trip
    -> LMMSE-CG equalisation of the data frames (Algorithm 1; otfs_lmmse_cg)
    -> hard decisions (Eq. demod) and, given the transmitted symbols, bit errors
       (otfs_bit_errors).

Argument marshalling only: every step runs in the library's kernels.  A packet is one
pilot frame and `ndata` data frames sharing one channel; the pilot's DD frame is
replicated on the device for the data frames of its packet.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import Plan, dzt


class _Placeholder:
    """Frame descriptor whose paths are placeholders: only the path capacity counts (the
    paths come from the pilot on the device)."""

    def __init__(self, M, N, cap, lam, qam):
        self.M, self.N = int(M), int(N)
        self.tau = np.zeros(cap, dtype=np.int32)
        self.nu = np.zeros(cap, dtype=np.int32)
        self.h = np.full(cap, 0.1, dtype=np.complex128)
        self.lam, self.qam = float(lam), int(qam)


def receive(ypilot_td, ydata_td, M: int, N: int, lam: float, qam: int, theta: float = 0.08,
            capacity: int = 64, max_iters: int = 10, rel_tol: float = 0.0,
            refresh_every: int = 0, sym_tx=None, stream=None):
    """ypilot_td: (npackets * M * N) complex64 cuda tensor, one received pilot per packet;
    ydata_td: (npackets * ndata * M * N) received data frames, packet after packet.
    Returns a dict: xhat, sym (decisions), stats, npaths (bins above theta per packet),
    plan, and errs (bit errors per data frame) when sym_tx is given."""
    import torch
    E = M * N
    npk = ypilot_td.numel() // E
    nd = ydata_td.numel() // E
    if npk < 1 or nd % npk or ypilot_td.numel() != npk * E or ydata_td.numel() != nd * E:
        raise ValueError("need npackets pilot frames and a multiple of them data frames")
    per = nd // npk
    yp_dd = dzt(ypilot_td, M, N, stream=stream)
    y_dd = dzt(ydata_td, M, N, stream=stream)
    pilots = yp_dd.view(npk, 1, E).expand(npk, per, E).reshape(-1).contiguous()
    plan = Plan([_Placeholder(M, N, capacity, lam, qam) for _ in range(nd)], max_iters=max_iters,
                rel_tol=rel_tol, refresh_every=refresh_every, tune=False)
    npaths = plan.paths_from_pilot(pilots, theta, stream=stream)
    sym = torch.empty(nd * E, dtype=torch.uint8, device="cuda")
    stats = plan.new_stats()
    xhat = plan.lmmse_cg(y_dd, sym=sym, stats=stats, stream=stream)
    out = {"xhat": xhat, "sym": sym, "stats": stats, "npaths": npaths[::per], "plan": plan,
           "y_dd": y_dd, "pilot_dd": yp_dd}
    if sym_tx is not None:
        out["errs"] = plan.bit_errors(sym, sym_tx, stream=stream)
    return out
