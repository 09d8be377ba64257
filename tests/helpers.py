"""Shared test helpers: oracle-side batch preparation and comparisons."""
import sys

import numpy as np

import oracle as O


def say(*a):
    """Name the case on stdout before a GPU step (flushed, so a crash still shows it)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


class SpecLike:
    def __init__(self, M, N, tau, nu, h, lam=0.01, qam=4):
        self.M, self.N = int(M), int(N)
        self.tau = np.asarray(tau, dtype=np.int32)
        self.nu = np.asarray(nu, dtype=np.int32)
        self.h = np.asarray(h, dtype=np.complex128)
        self.lam, self.qam = float(lam), int(qam)

    @property
    def P(self):
        return int(self.tau.shape[0])

    @property
    def E(self):
        return self.M * self.N


def oracle_batch(frames):
    """Per-frame oracle operators, transmitted symbols and received frames (complex64),
    concatenated in batch order."""
    ops, xs, ys = [], [], []
    for fr in frames:
        op, x, y = O.received_frame(fr)
        ops.append(op)
        xs.append(x)
        ys.append(y)
    return ops, xs, np.concatenate(ys).astype(np.complex64)


def iters_close(it_gpu, it_ref, capped):
    """Stop iteration of the FP32 solve vs the FP64 oracle under the same rule.  Capped
    runs stop at the same count.  Otherwise the two follow different rounding paths and
    a relative residual of 1e-6 is near what FP32 CG attains, so the FP32 run may stop a
    few iterations later (or one earlier): allow max(1, 10 %) of the oracle's count."""
    if capped:
        return it_gpu == it_ref
    return abs(int(it_gpu) - int(it_ref)) <= max(1, int(it_ref) // 10)


def split(v, frames):
    out, o = [], 0
    for fr in frames:
        E = fr.spec.E if hasattr(fr, "spec") else fr.E
        out.append(v[o:o + E])
        o += E
    return out


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def check_decisions(sym_gpu, x_gpu, x_ref, Q, delta=1e-3):
    """Decisions of the GPU equal (a) the decision rule applied in FP32 to the GPU's own
    estimate, bit for bit, and (b) the FP64 oracle's decisions wherever the oracle's
    estimate is farther than delta from a decision boundary; nearer points may take
    either neighbouring level.  Returns the number of such ambiguous symbols."""
    sym_gpu = np.asarray(sym_gpu, dtype=np.uint8)
    own = O.qam_decide(np.asarray(x_gpu, dtype=np.complex64), Q, np.float32)
    assert np.array_equal(sym_gpu, own), "decision step differs from the FP32 rule"
    ref = O.qam_decide(x_ref, Q)
    safe = O.decision_margin(x_ref, Q) > delta
    bad = np.nonzero((sym_gpu != ref) & safe)[0]
    assert bad.size == 0, f"{bad.size} decisions differ away from boundaries"
    m = O.qam_side(Q)
    amb = ~safe
    d_i = np.abs(sym_gpu[amb].astype(int) // m - ref[amb].astype(int) // m)
    d_q = np.abs(sym_gpu[amb].astype(int) % m - ref[amb].astype(int) % m)
    assert np.all(d_i <= 1) and np.all(d_q <= 1)
    return int(amb.sum())
