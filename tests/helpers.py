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


# Rounding allowance of a decision taken in FP32 (signal units): the oracle's estimate
# rounded to complex64 moves by at most 2^-24 |x| (< 1.2e-7 for |x| < 2), and the FP32 rule
# t = ((v s) + m) / 2 errs by at most two ulps of t <= m, which is 2 ulp(m) * 2 / s in
# signal units: 3.4e-7 (QPSK), 6.0e-7 (16-QAM), 5.9e-7 (64-QAM), 5.8e-7 (256-QAM).  The sum
# stays below 2^-20 = 9.5e-7.
DECISION_FP32_SLACK = 2.0 ** -20


def check_decisions(sym_gpu, x_gpu, x_ref, Q):
    """Hard decisions of the GPU against the oracle's (Eq. demod), both taken in the
    kernel's precision (the FP32 rule), the oracle's on its FP64 estimate rounded to
    complex64.

    (a) The GPU's decisions equal the FP32 rule applied to the GPU's own estimate, bit for
        bit.
    (b) Wherever they differ from the oracle's, the difference is explained by the
        estimates themselves: the oracle's estimate lies closer to a decision boundary than
        the GPU's estimate lies to the oracle's, up to the FP32 rounding allowance
        (margin(x_ref) < |x_gpu - x_ref| + DECISION_FP32_SLACK), so the GPU's point can sit
        on the other side.  A decision that differs with a larger margin fails.
    Returns the number of decisions that differ from the oracle's (all of them explained).
    """
    sym_gpu = np.asarray(sym_gpu, dtype=np.uint8)
    x_gpu = np.asarray(x_gpu)
    own = O.qam_decide(x_gpu.astype(np.complex64), Q, np.float32)
    assert np.array_equal(sym_gpu, own), "decision step differs from the FP32 rule"
    ref = O.qam_decide(np.asarray(x_ref).astype(np.complex64), Q, np.float32)
    diff = np.nonzero(sym_gpu != ref)[0]
    if diff.size:
        margin = O.decision_margin(x_ref[diff], Q)
        err = np.abs(x_gpu[diff].astype(np.complex128) - x_ref[diff])
        bad = diff[margin >= err + DECISION_FP32_SLACK]
        assert bad.size == 0, (f"{bad.size} of {diff.size} differing decisions lie farther from "
                               f"a boundary than the estimate error (first at {bad[0]})")
    return int(diff.size)


def ser(sym, sym_tx):
    """Symbol error rate of hard decisions against the transmitted indices."""
    return float(np.mean(np.asarray(sym, dtype=np.int64) != np.asarray(sym_tx, dtype=np.int64)))


def bf16_round(a):
    """complex64 values rounded to bf16 per component, round to nearest even (the rounding
    torch.Tensor.to(torch.bfloat16) performs): returns (uint16 bits (re, im interleaved),
    the rounded values as complex64).  Inputs are finite."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.complex64)).view(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    bits = u.astype(np.uint16)
    back = (bits.astype(np.uint32) << 16).view(np.float32).view(np.complex64)
    return bits, back


# ----------------------------------------------------------------------------------------
# Oracle jobs for a process pool (module level so they can be pickled).  Workers run NumPy
# only; they never touch the GPU.
# ----------------------------------------------------------------------------------------
def oracle_received(frame):
    """(y rounded to complex64, transmitted symbol indices) of a workload frame."""
    _, _, y = O.received_frame(frame)
    return y, np.asarray(frame.sym)


def oracle_solve(args):
    """FP64 CG (the identical stop rule) of one frame.  args = (frame, y or None): y None
    uses the frame's own received y.  Returns (y, x_ref, iters, rel_res)."""
    frame, y = args
    sp = frame.spec
    op = O.TwistedConvChannel(sp.M, sp.N, sp.h, sp.tau, sp.nu)
    if y is None:
        _, _, y = O.received_frame(frame)
    x, it, rel = O.cg_lmmse(y, op, sp.lam, sp.max_iters, sp.tol)
    return y, x, it, rel


def pool_map(pool, fn, jobs, label, every=16):
    """pool.imap in order, printing progress so a long oracle phase is never silent."""
    out = []
    for i, r in enumerate(pool.imap(fn, jobs, chunksize=1)):
        out.append(r)
        if (i + 1) % every == 0 or i + 1 == len(jobs):
            say(label, f"{i + 1}/{len(jobs)} oracle frames")
    return out
