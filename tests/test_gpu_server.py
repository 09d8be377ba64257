"""GPU tests of the serving loop through the C ABI: frames that arrive over time, run in
steps of a few CG iterations among whatever else is admitted, match the FP64 oracle, and
give the same bits alone, among other frames, and through a plan of the same tiling."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import check_decisions, iters_close, say, to_dev

pytestmark = pytest.mark.gpu

NMSE_TOL = 1e-5
MAX_ITERS, TOL = 50, 1e-6
SERVE_TILE_ELEMS = 32768     # the server's frame-local tiling rule


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _frames(seed, n, shapes=((64, 16), (128, 32), (96, 24), (512, 128), (37, 11))):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M, N = shapes[i % len(shapes)]
        P = int(rng.integers(2, 7))
        out.append(W.small_frame(rng, M, N, P, (0, min(12, M - 1)),
                                 (-min(6, N - 1), min(6, N - 1)),
                                 qam=(4, 16, 64)[i % 3], snr_db=float(rng.uniform(8, 30)),
                                 max_iters=MAX_ITERS, tol=TOL))
    return out


def _serve(srv, frames, ys):
    tickets = [srv.submit(fr.spec, y) for fr, y in zip(frames, ys)]
    return [srv.wait(t, fr.spec, timeout=60.0) for t, fr in zip(tickets, frames)]


def test_server_matches_oracle_and_plan(otfs):
    import torch
    frames = _frames(11, 10)
    ops, ys = [], []
    for fr in frames:
        op, _, y = O.received_frame(fr)
        ops.append(op)
        ys.append(np.asarray(y, np.complex64))
    say("server vs oracle", [(f.spec.M, f.spec.N, f.spec.P) for f in frames])
    with otfs.Server(256 << 20, max_iters=MAX_ITERS, rel_tol=TOL, step_iters=7, tune=False) as srv:
        res = _serve(srv, frames, ys)
        ss = srv.stats()
    assert ss.completed == len(frames) and ss.pool_bytes_in_use == 0
    for i, (fr, (x, sym, st, lat)) in enumerate(zip(frames, res)):
        sp = fr.spec
        xr, it_r, rel_r = O.cg_lmmse(ys[i].astype(np.complex128), ops[i], sp.lam,
                                     MAX_ITERS, TOL)
        nm = O.nmse(x, xr)
        assert nm <= NMSE_TOL, f"frame {i} ({sp.M}x{sp.N}): NMSE {nm:.3e}"
        assert st.status in (otfs.FRAME_CONVERGED, otfs.FRAME_CAPPED)
        assert iters_close(st.iters, it_r, rel_r > TOL * 1.5 and it_r == MAX_ITERS)
        assert lat > 0
        check_decisions(sym, x, xr, sp.qam)
    # the same frame through a plan with the server's tiling gives the same bits
    for i in (0, 3):
        fr = frames[i]
        plan = otfs.Plan([fr.spec], max_iters=MAX_ITERS, rel_tol=TOL,
                         tile_elems=SERVE_TILE_ELEMS)
        sym = torch.zeros(fr.spec.E, dtype=torch.uint8, device="cuda")
        xp = plan.lmmse_cg(to_dev(ys[i]), sym=sym)
        torch.cuda.synchronize()
        assert np.array_equal(xp.cpu().numpy().view(np.uint32), res[i][0].view(np.uint32)), i
        assert np.array_equal(sym.cpu().numpy(), res[i][1]), i


def test_server_alone_equals_in_mix(otfs):
    frames = _frames(12, 16)
    ys = [np.asarray(O.received_frame(fr)[2], np.complex64) for fr in frames]
    target = 3
    say("server alone vs mix, target", frames[target].spec.M, frames[target].spec.N)
    with otfs.Server(512 << 20, max_iters=MAX_ITERS, rel_tol=TOL, step_iters=5) as srv:
        alone = _serve(srv, [frames[target]], [ys[target]])[0]
        mix = _serve(srv, frames, ys)[target]
    assert np.array_equal(alone[0].view(np.uint32), mix[0].view(np.uint32))
    assert np.array_equal(alone[1], mix[1])
    assert alone[2].iters == mix[2].iters and alone[2].status == mix[2].status


def test_server_kind_switch_keeps_bits(otfs):
    # A frame with few paths runs the kind that forms the direction inside the H gathers
    # while it is alone; next to a 12-path frame the steps use the split form. Both forms
    # compute the same values in the same order, so its result is the same bits.
    frames = _frames(14, 1, shapes=((128, 32),))
    rng = np.random.default_rng(15)
    frames.append(W.small_frame(rng, 256, 16, 12, (0, 12), (-6, 6), qam=16, snr_db=20.0,
                                max_iters=MAX_ITERS, tol=TOL))
    ys = [np.asarray(O.received_frame(fr)[2], np.complex64) for fr in frames]
    say("server kind switch", [(f.spec.M, f.spec.N, f.spec.P) for f in frames])
    with otfs.Server(256 << 20, max_iters=MAX_ITERS, rel_tol=TOL, step_iters=4) as srv:
        alone = _serve(srv, frames[:1], ys[:1])[0]
        mix = _serve(srv, frames, ys)
    assert np.array_equal(alone[0].view(np.uint32), mix[0][0].view(np.uint32))
    assert np.array_equal(alone[1], mix[0][1])
    assert alone[2].iters == mix[0][2].iters
    xr, _, _ = O.cg_lmmse(ys[1].astype(np.complex128), O.received_frame(frames[1])[0],
                          frames[1].spec.lam, MAX_ITERS, TOL)
    assert O.nmse(mix[1][0], xr) <= NMSE_TOL


def test_server_under_pool_pressure(otfs):
    frames = _frames(13, 8, shapes=((128, 32),))
    ys = [np.asarray(O.received_frame(fr)[2], np.complex64) for fr in frames]
    with otfs.Server(64 << 20, device=-1) as probe:
        fb, cb = probe.frame_bytes(frames[0].spec)
    say("server pool pressure: two frames at a time", fb, cb)
    with otfs.Server(cb + 2 * fb + 1024, max_iters=MAX_ITERS, rel_tol=TOL,
                     step_iters=3) as srv:
        res = _serve(srv, frames, ys)
        ss = srv.stats()
    assert ss.completed == 8 and ss.pool_bytes_peak <= 2 * fb
    with otfs.Server(256 << 20, max_iters=MAX_ITERS, rel_tol=TOL, step_iters=50) as srv:
        ref = _serve(srv, frames, ys)
    for a, b in zip(res, ref):
        assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


def test_server_refresh_matches_plan(otfs):
    # With the FP64 true-residual refresh every 5 iterations and steps of 7, frames reach
    # their refresh points in the middle of a step; they wait for the refresh launches at
    # the end of the step and resume in the next one.  Each result equals, bit for bit, the
    # same frame solved by a plan with the server's tiling and the same refresh period.
    import torch
    frames = _frames(16, 5)
    ys = [np.asarray(O.received_frame(fr)[2], np.complex64) for fr in frames]
    say("server with refresh every 5", [(f.spec.M, f.spec.N, f.spec.P) for f in frames])
    with otfs.Server(256 << 20, max_iters=MAX_ITERS, rel_tol=TOL, refresh_every=5, tune=False,
                     step_iters=7) as srv:
        res = _serve(srv, frames, ys)
    for i, fr in enumerate(frames):
        sp = fr.spec
        xr, _, _ = O.cg_lmmse(ys[i].astype(np.complex128), O.received_frame(fr)[0], sp.lam,
                              MAX_ITERS, TOL)
        assert O.nmse(res[i][0], xr) <= NMSE_TOL, i
        plan = otfs.Plan([sp], max_iters=MAX_ITERS, rel_tol=TOL, refresh_every=5,
                         tile_elems=SERVE_TILE_ELEMS)
        sym = torch.zeros(sp.E, dtype=torch.uint8, device="cuda")
        stats = plan.new_stats()
        xp = plan.lmmse_cg(to_dev(ys[i]), sym=sym, stats=stats)
        torch.cuda.synchronize()
        assert np.array_equal(xp.cpu().numpy().view(np.uint32), res[i][0].view(np.uint32)), i
        assert np.array_equal(sym.cpu().numpy(), res[i][1]), i
        assert int(otfs.stats_numpy(stats)["iters"][0]) == res[i][2].iters
