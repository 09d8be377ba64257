"""GPU parity of the structured-sparse channel built on the device from a received pilot
frame (otfs_plan_paths_from_pilot) against the FP64 oracle.

The pilot (one impulse at (M/2, N/2)) goes through a channel with strong paths, weak paths
below the threshold and noise; the oracle estimates the channel on the received grid
(Eq. heff_hadamard) and thresholds it (Eq. heff_thres, theta = 0.08, the decision in FP32 as
the kernel takes it).  The device path set must equal the oracle's exactly (count, and the
operator built from it applied element by element within FP32 tolerance), and the
equaliser driven by the device-built channel must match the oracle's CG run with the
oracle's estimate (NMSE <= 1e-5)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import SpecLike, say, split, to_dev

pytestmark = pytest.mark.gpu

THETA = 0.08      # Sec. VI-A
NMSE_TOL = 1e-5


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _channel(rng, M, N, strong, weak):
    """Distinct bins inside the estimate's support (|tau| < M/2, |nu| < N/2): `strong` paths
    with |h| in [0.15, 1], `weak` ones with |h| < 0.04 (below theta)."""
    P = strong + weak
    n_t, n_v = M - 1, N - 1
    pick = rng.choice(n_t * n_v, size=P, replace=False)
    tau = pick // n_v - (M // 2 - 1)
    nu = pick % n_v - (N // 2 - 1)
    ph = np.exp(2j * np.pi * rng.uniform(0, 1, P))
    mag = np.concatenate([rng.uniform(0.15, 1.0, strong), rng.uniform(0.0, 0.04, weak)])
    return tau.astype(np.int32), nu.astype(np.int32), mag * ph


def _pilot_batch(seed, shapes, cap, snr_db=35.0, data_snr_db=20.0):
    """Pilot frames at snr_db (clean detection); the data frames' noise and the equaliser's
    lam at data_snr_db."""
    rng = np.random.default_rng(seed)
    cases = []
    for i, (M, N) in enumerate(shapes):
        tau, nu, h = _channel(rng, M, N, strong=3 + i % 5, weak=2)
        lam_p = 10.0 ** (-snr_db / 10.0)
        lam = 10.0 ** (-data_snr_db / 10.0)
        op = O.TwistedConvChannel(M, N, h, tau, nu)
        w = math.sqrt(lam_p / 2.0) * (rng.standard_normal(M * N) + 1j * rng.standard_normal(M * N))
        yp = (op.apply(O.pilot_frame(M, N)) + w).astype(np.complex64)
        est = O.pilot_estimate_hadamard(yp.astype(np.complex128), M, N)
        t_o, v_o, g_o = O.threshold_paths(est, THETA, np.float32)
        count = t_o.size
        t_o, v_o, g_o = t_o[:cap], v_o[:cap], g_o[:cap]     # the capacity keeps the first
        # placeholder paths: the capacity only (replaced on the device)
        ph = SpecLike(M, N, [0] * cap, [0] * cap, [0.1] * cap, lam=lam, qam=16)
        cases.append(dict(M=M, N=N, true=(tau, nu, h), yp=yp, ref=(t_o, v_o, g_o), count=count, ph=ph,
                          lam=lam, rng_x=rng.standard_normal(2 * M * N)))
    return cases


def _rand_c(rng, n):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)


@pytest.mark.parametrize("flags,refresh", [(0, 0), ("stored_c64", 10)])
def test_pilot_paths_match_oracle(otfs, flags, refresh):
    import torch
    shapes = [(64, 16), (128, 32), (96, 24), (256, 64), (37, 11)]
    cap = 12
    cases = _pilot_batch(21, shapes, cap)
    fl = otfs.D_STORED_C64 if flags == "stored_c64" else 0
    say("pilot paths", shapes, "flags", fl, "refresh", refresh)
    plan = otfs.Plan([c["ph"] for c in cases], refresh_every=refresh, flags=fl)
    yp = to_dev(np.concatenate([c["yp"] for c in cases]))
    npaths = plan.paths_from_pilot(yp, THETA)
    torch.cuda.synchronize()
    npaths = npaths.cpu().numpy()
    for c, n in zip(cases, npaths):
        assert int(n) == c["count"], (c["M"], c["N"], int(n), c["count"])
    # the operator built on the device against the oracle's operator of its own estimate
    rng = np.random.default_rng(5)
    E = plan.total_elems
    x = _rand_c(rng, E)
    y = _rand_c(rng, E)
    yh = plan.apply_H(to_dev(x)).cpu().numpy()
    xh = plan.apply_HH(to_dev(y)).cpu().numpy()
    o = 0
    for c in cases:
        M, N = c["M"], c["N"]
        t_o, v_o, g_o = c["ref"]
        op = O.TwistedConvChannel(M, N, g_o, t_o, v_o)
        sl = slice(o, o + M * N)
        scale = max(np.abs(g_o).sum(), 1e-3)
        assert np.abs(yh[sl] - op.apply(x[sl].astype(np.complex128))).max() <= \
            2e-5 * scale * np.abs(x[sl]).max(), (M, N)
        assert np.abs(xh[sl] - op.apply_adjoint(y[sl].astype(np.complex128))).max() <= \
            2e-5 * scale * np.abs(y[sl]).max(), (M, N)
        o += M * N
    # equalisation of data frames through the true channel, with the estimated one
    xs, ys, ops = [], [], []
    for c in cases:
        M, N = c["M"], c["N"]
        tau, nu, h = c["true"]
        sym = np.random.default_rng(M * N).integers(0, 16, M * N)
        xt = O.qam_points(sym, 16)
        w = math.sqrt(c["lam"] / 2.0) * (c["rng_x"][:M * N] + 1j * c["rng_x"][M * N:])
        ys.append((O.TwistedConvChannel(M, N, h, tau, nu).apply(xt) + w).astype(np.complex64))
        t_o, v_o, g_o = c["ref"]
        ops.append(O.TwistedConvChannel(M, N, g_o, t_o, v_o))
    sym_d = torch.zeros(E, dtype=torch.uint8, device="cuda")
    xg = plan.lmmse_cg(to_dev(np.concatenate(ys)), sym=sym_d).cpu().numpy()
    for i, c in enumerate(cases):
        xr, _, _ = O.cg_lmmse(ys[i].astype(np.complex128), ops[i], c["lam"], 50, 1e-6)
        nm = O.nmse(split(xg, [c["ph"] for c in cases])[i], xr)
        assert nm <= NMSE_TOL, (c["M"], c["N"], nm)


def test_pilot_paths_capacity_keeps_first_in_vector_order(otfs):
    import torch
    # a noisy pilot (10 dB) puts many bins above theta; capacity 4 keeps the first four in
    # vector order, and the count reports all of them
    cases = _pilot_batch(33, [(64, 16), (128, 32)], cap=4, snr_db=10.0)
    say("pilot paths, capacity 4")
    plan = otfs.Plan([c["ph"] for c in cases])
    yp = to_dev(np.concatenate([c["yp"] for c in cases]))
    npaths = plan.paths_from_pilot(yp, THETA).cpu().numpy()
    rng = np.random.default_rng(9)
    E = plan.total_elems
    x = _rand_c(rng, E)
    yh = plan.apply_H(to_dev(x)).cpu().numpy()
    o = 0
    for c, n in zip(cases, npaths):
        M, N = c["M"], c["N"]
        t_o, v_o, g_o = c["ref"]
        assert int(n) == c["count"] and c["count"] > 4 and t_o.size == 4
        op = O.TwistedConvChannel(M, N, g_o, t_o, v_o)
        sl = slice(o, o + M * N)
        assert np.abs(yh[sl] - op.apply(x[sl].astype(np.complex128))).max() <= \
            2e-5 * np.abs(g_o).sum() * np.abs(x[sl]).max()
        o += M * N
