"""LDS-windowed paired gathers (OTFS_LDS_GATHER): the fused solve of multi-tile frames whose
rows split into 16-byte pairs reads each strip's source window once into LDS and gathers
every path from there.  It must give the same bits as the direct paired gathers (the same
sums in the same order, Algorithm 1 unchanged) and match the oracle (NMSE <= 1e-5).  The
cases cover windows inside the frame, windows that span every row (Doppler range plus band
at least N) or every column (delay range plus strip at least M), negative delays, delay
and Doppler wraps, ragged bands, and the FP64 refresh between fused segments."""
import numpy as np
import pytest

import oracle as O
from helpers import SpecLike, say, to_dev

pytestmark = pytest.mark.gpu
NMSE_TOL = 1e-5


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _frames(rng, M, N, P, tau_rng, nu_rng, n, qam=16, snr_db=25.0):
    out = []
    for _ in range(n):
        pairs = set()
        while len(pairs) < P:
            pairs.add((int(rng.integers(tau_rng[0], tau_rng[1] + 1)),
                       int(rng.integers(nu_rng[0], nu_rng[1] + 1))))
        pairs = sorted(pairs)
        h = (rng.standard_normal(P) + 1j * rng.standard_normal(P)) / np.sqrt(2 * P)
        out.append(SpecLike(M, N, [p[0] for p in pairs], [p[1] for p in pairs], h,
                            lam=10 ** (-snr_db / 10), qam=qam))
    return out


def _received(rng, frames):
    ops, ys = [], []
    for f in frames:
        op = O.TwistedConvChannel(f.M, f.N, f.h, f.tau, f.nu)
        x = O.qam_points(rng.integers(0, f.qam, f.E), f.qam)
        w = np.sqrt(f.lam / 2) * (rng.standard_normal(f.E) + 1j * rng.standard_normal(f.E))
        ops.append(op)
        ys.append((op.apply(x) + w).astype(np.complex64))
    return ops, ys


CASES = [
    # M, N, P, delays, Dopplers, tile elements, refresh
    (1024, 64, 6, (0, 16), (-4, 4), 32768, 0),          # window inside the frame, 2 tiles
    (1024, 64, 8, (-9, 20), (-6, 5), 21846, 0),         # negative delays, ragged bands (22/21/21)
    (128, 64, 6, (0, 127), (-5, 5), 1024, 0),           # delay range spans the row: all columns
    (1024, 32, 6, (0, 12), (-8, 8), 16384, 0),          # Doppler range spans the frame: all rows
    (1024, 64, 16, (0, 64), (-16, 16), 16384, 0),       # the headline's path count and ranges
    (512, 32, 10, (0, 40), (-10, 10), 4096, 3),         # with the FP64 refresh every 3
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lds_gather_same_bits_as_direct(otfs, case):
    import torch
    M, N, P, tr, vr, te, ref = CASES[case]
    rng = np.random.default_rng(9100 + case)
    frames = _frames(rng, M, N, P, tr, vr, 5)
    ops, ys = _received(rng, frames)
    y = to_dev(np.concatenate(ys))
    say("lds gather case", case, (M, N, P, tr, vr, te, ref))
    res = {}
    for name, fl in (("direct", otfs.SPLIT_DIRECTION), ("lds", otfs.LDS_GATHER)):
        plan = otfs.Plan(frames, max_iters=30, rel_tol=1e-6, refresh_every=ref, flags=fl,
                         tile_elems=te, tune=False)
        info = plan.info()
        if name == "lds":
            assert info.staged_frames == len(frames), "every frame takes the LDS windows"
            assert info.lds_bytes > 0
        else:
            assert info.staged_frames == 0
        st = plan.new_stats()
        sym = torch.zeros(y.numel(), dtype=torch.uint8, device="cuda")
        x = plan.lmmse_cg(y, sym=sym, stats=st)
        torch.cuda.synchronize()
        res[name] = (x.cpu().numpy(), sym.cpu().numpy(), otfs.stats_numpy(st))
        del plan
    xd, sd, std = res["direct"]
    xl, sl, stl = res["lds"]
    assert np.array_equal(xd.view(np.uint32), xl.view(np.uint32))
    assert np.array_equal(sd, sl)
    assert np.array_equal(std, stl)
    o = 0
    worst = 0.0
    for f, op, yy in zip(frames, ops, ys):
        xr, _, _ = O.cg_lmmse(yy.astype(np.complex128), op, f.lam, 30, 1e-6)
        nm = O.nmse(xl[o:o + f.E], xr)
        worst = max(worst, nm)
        assert nm <= NMSE_TOL, nm
        o += f.E
    say(f"case {case}: bit-identical to the direct gathers; worst NMSE vs oracle {worst:.2e}")


@pytest.mark.parametrize("cover", [False, True])
def test_lds_gather_device_paths_with_refresh(otfs, cover):
    """Path tables made on the device from a pilot (Eqs. heff_hadamard, heff_thres) with the
    FP64 refresh every 3 iterations.  With placeholder paths whose ranges cover the estimated
    ones the windows fit and those frames refresh inside the fused launch: the same bits as
    the direct gathers.  With all-zero placeholders the estimated ranges outgrow the planned
    windows, so the gathers read memory one element per lane (their partial sums then add
    in another order than the direct kind's pairs) and the frames refresh in the refresh
    launches.  Either way every frame finishes its fixed iteration count and the oracle's
    solve with the device's path table agrees (NMSE <= 1e-5)."""
    import torch
    M, N, P, cap, theta = 256, 32, 6, 8, 0.08
    rng = np.random.default_rng(9300 + int(cover))
    frames = _frames(rng, M, N, P, (0, 12), (-4, 4), 4)
    for f in frames:   # gains well above the threshold
        f.h = 0.5 * np.exp(2j * np.pi * rng.random(P))
    ops, ys = _received(rng, frames)
    yp = []
    for f, op in zip(frames, ops):
        w = 1e-3 * (rng.standard_normal(f.E) + 1j * rng.standard_normal(f.E))
        yp.append((op.apply(O.pilot_frame(M, N)) + w).astype(np.complex64))
    if cover:
        tau_ph = [0, 12] + [0] * (cap - 2)
        nu_ph = [-4, 4] + [0] * (cap - 2)
    else:
        tau_ph, nu_ph = [0] * cap, [0] * cap
    ph = [SpecLike(M, N, tau_ph, nu_ph, [0.1] * cap, lam=f.lam, qam=f.qam) for f in frames]
    y = to_dev(np.concatenate(ys))
    ypd = to_dev(np.concatenate(yp))
    say("lds gather, device paths, cover", cover)
    res = {}
    for name, fl in (("direct", otfs.SPLIT_DIRECTION), ("lds", otfs.LDS_GATHER)):
        plan = otfs.Plan(ph, max_iters=20, rel_tol=0.0, refresh_every=3, flags=fl,
                         tile_elems=2048, tune=False)
        n = plan.paths_from_pilot(ypd, theta).cpu().numpy()
        assert np.all(n == P), n
        st = plan.new_stats()
        sym = torch.zeros(y.numel(), dtype=torch.uint8, device="cuda")
        x = plan.lmmse_cg(y, sym=sym, stats=st)
        torch.cuda.synchronize()
        paths = [plan.get_paths(i) for i in range(len(frames))]
        res[name] = (x.cpu().numpy(), sym.cpu().numpy(), otfs.stats_numpy(st), paths)
        del plan
    xd, sd, std, pd = res["direct"]
    xl, sl, stl, pl = res["lds"]
    for a, b in zip(pd, pl):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    if cover:
        assert np.array_equal(xd.view(np.uint32), xl.view(np.uint32))
        assert np.array_equal(sd, sl)
        assert np.array_equal(std, stl)
    else:
        assert O.nmse(xl, xd.astype(np.complex128)) <= 1e-9
    for st in (std, stl):
        assert np.all(st["status"] == otfs.FRAME_CAPPED), st["status"]
        assert np.all(st["iters"] == 20)
    o = 0
    worst = 0.0
    for i, (f, yy) in enumerate(zip(frames, ys)):
        t, v, g = pl[i]
        op = O.TwistedConvChannel(M, N, g.astype(np.complex128), t, v)
        xr, _, _ = O.cg_lmmse(yy.astype(np.complex128), op, f.lam, 20, 0.0)
        nm = O.nmse(xl[o:o + f.E], xr)
        worst = max(worst, nm)
        assert nm <= NMSE_TOL, nm
        o += f.E
    say(f"device paths (cover={cover}): worst NMSE vs oracle {worst:.2e}")
