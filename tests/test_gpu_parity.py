"""GPU parity of libotfs against the FP64 oracle, through the C ABI.

Inputs are seeded and synthetic; every received frame y is produced by the oracle
(complex128, rounded once to complex64) and the GPU consumes exactly that y.  Operator
applications are compared element by element; CG estimates per frame by NMSE <= 1e-5
against the oracle's CG run under the identical stop rule; hard decisions bit-exactly
(see helpers.check_decisions).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import SpecLike, check_decisions, iters_close, oracle_batch, say, split, to_dev

pytestmark = pytest.mark.gpu

NMSE_TOL = 1e-5          # FP32 path vs FP64 oracle, per frame
NMSE_TOL_BF16 = 1e-4     # y and D stored as bf16


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _rand_c(rng, n):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)


# every wrap case of the operator: tau at 0 and M-1, negative tau, nu at +-(N-1),
# M or N equal to one, sizes that are not powers of two, frames wider than a workgroup
EDGE_FRAMES = [
    (8, 4, [0, 7, -3, 2, 1, 0], [0, 3, -2, -3, 1, 2]),
    (5, 3, [4, -4, 2], [2, -2, 1]),
    (1, 4, [0, 0], [3, -3]),
    (6, 1, [5, -5, 2], [0, 0, 0]),
    (7, 5, [6, -6, 0, 3], [-4, 4, 0, -1]),
    (64, 16, [0, 8, 63, -63], [0, -4, 15, -15]),
    (100, 30, [0, 99, -50, 17], [29, -29, 3, 0]),
    (300, 12, [299, -1, 150], [11, -11, 5]),
    (256, 64, list(range(0, 16)), list(range(-8, 8))),
    (1, 1, [0], [0]),
]


def _edge_specs(rng):
    out = []
    for M, N, tau, nu in EDGE_FRAMES:
        h = _rand_c(rng, len(tau)).astype(np.complex128) / math.sqrt(len(tau))
        out.append(SpecLike(M, N, tau, nu, h, lam=0.02, qam=16))
    return out


@pytest.mark.parametrize("tile_elems,stage", [(0, None), (64, None), (1024, None), (0, 0),
                                              (1024, 16384), (64, 65536)])
def test_apply_parity_edge_batch(otfs, tile_elems, stage):
    rng = np.random.default_rng(7 + tile_elems)
    specs = _edge_specs(rng)
    say("apply parity", "tile_elems", tile_elems, "stage", stage, [(s.M, s.N, s.P) for s in specs])
    plan = otfs.Plan(specs, tile_elems=tile_elems, stage_bytes=stage)
    say("  lds_bytes", plan.info().lds_bytes)
    E = plan.total_elems
    x = _rand_c(rng, E)
    y = _rand_c(rng, E)
    yh = plan.apply_H(to_dev(x)).cpu().numpy()
    xh = plan.apply_HH(to_dev(y)).cpu().numpy()
    o = 0
    for s in specs:
        op = O.TwistedConvChannel(s.M, s.N, s.h, s.tau, s.nu)
        sl = slice(o, o + s.E)
        ref_f = op.apply(x[sl].astype(np.complex128))
        ref_a = op.apply_adjoint(y[sl].astype(np.complex128))
        scale = np.abs(s.h).sum()
        assert np.abs(yh[sl] - ref_f).max() <= 1e-5 * scale * np.abs(x[sl]).max(), (s.M, s.N)
        assert np.abs(xh[sl] - ref_a).max() <= 1e-5 * scale * np.abs(y[sl]).max(), (s.M, s.N)
        o += s.E


def _cg_check(plan_out, frames, ops, y, tol_nmse, form="fused"):
    xg, symg, stg = plan_out
    xs = split(xg, frames)
    syms = split(symg, frames)
    ys = split(y, frames)
    amb_total = 0
    for i, fr in enumerate(frames):
        sp = fr.spec
        xr, it_r, rel_r = O.cg_lmmse(ys[i], ops[i], sp.lam, sp.max_iters, sp.tol)
        nm = O.nmse(xs[i], xr)
        assert nm <= tol_nmse, f"{form} frame {i} ({sp.M}x{sp.N}, P={sp.P}): NMSE {nm:.3e}"
        it_g = int(stg["iters"][i])
        capped = rel_r > sp.tol * 1.5 and it_r == sp.max_iters
        assert iters_close(it_g, it_r, capped), (i, it_g, it_r)
        assert stg["status"][i] in (O_CONV, O_CAP)
        amb_total += check_decisions(syms[i], xs[i], xr, sp.qam)
    return amb_total


O_CONV, O_CAP = 1, 2


def _run(otfs, plan, y, form="fused"):
    import torch
    yd = to_dev(y)
    sym = torch.zeros(plan.total_elems, dtype=torch.uint8, device="cuda")
    stats = plan.new_stats()
    fn = plan.lmmse_cg if form == "fused" else plan.lmmse_cg_plain
    x = fn(yd, sym=sym, stats=stats)
    torch.cuda.synchronize()
    return x.cpu().numpy(), sym.cpu().numpy(), otfs.stats_numpy(stats)


def _mixed_frames(seed, n, shapes, P_range, tau_max, nu_max, qams=(4, 16), snr=(10, 30),
                  max_iters=50, tol=1e-6):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M, N = shapes[i % len(shapes)]
        P = int(rng.integers(P_range[0], P_range[1] + 1))
        fr = W.small_frame(rng, M, N, P, (0, min(tau_max, M - 1)),
                           (-min(nu_max, N - 1), min(nu_max, N - 1)),
                           qam=int(qams[i % len(qams)]),
                           snr_db=float(rng.uniform(*snr)), max_iters=max_iters, tol=tol)
        out.append(fr)
    return out


def test_cg_single_64x16_config(otfs):
    fr = W.draw_frame("single_64x16", 0)
    frames = [fr]
    ops, xs, y = oracle_batch(frames)
    for form in ("fused", "plain"):
        say("cg single_64x16", form)
        plan = otfs.Plan([fr.spec], max_iters=30, rel_tol=1e-6)
        _cg_check(_run(otfs, plan, y, form), frames, ops, y, NMSE_TOL, form)


@pytest.mark.parametrize("tile_elems,max_grid,agent,stage", [
    (0, 0, 0, None), (700, 0, 0, None), (700, 8, 1, None), (700, 64, 0, None),
    (2048, 3, 1, None), (0, 0, 1, None), (350, 0, 0, None), (200, 0, 0, None),
    (200, 0, 1, None), (0, 0, 0, 0), (700, 0, 0, 0), (700, 0, 0, 16384), (700, 0, 0, 40960),
    (0, 0, 1, 40960)])
def test_cg_ragged_batch_tilings(otfs, tile_elems, max_grid, agent, stage):
    frames = _mixed_frames(11, 9, [(128, 32), (64, 16), (100, 30), (96, 8), (256, 16)],
                           (1, 9), 12, 4)
    ops, xs, y = oracle_batch(frames)
    say("cg ragged", tile_elems, max_grid, "agent" if agent else "xcd", "stage", stage)
    plan = otfs.Plan([f.spec for f in frames], tile_elems=tile_elems, max_grid=max_grid,
                     flags=otfs.AGENT_BARRIER if agent else 0, stage_bytes=stage)
    inf = plan.info()
    say("  groups", inf.groups, "xcd_local", inf.xcd_local, "grid", inf.grid)
    if agent:
        assert inf.groups == 1 and inf.xcd_local == 0
    _cg_check(_run(otfs, plan, y), frames, ops, y, NMSE_TOL)


def test_cg_resident_small_frames(otfs):
    # one-tile frames whose vectors fit in LDS run the resident form; with
    # NO_LDS_RESIDENT the same frames run the memory form
    frames = _mixed_frames(21, 8, [(64, 16), (32, 32), (37, 11), (8, 4), (5, 3), (16, 64),
                                   (1, 7), (100, 10)], (1, 6), 12, 4)
    ops, xs, y = oracle_batch(frames)
    say("cg resident small frames", [(f.spec.M, f.spec.N, f.spec.P) for f in frames])
    res = otfs.Plan([f.spec for f in frames])
    assert res.info().resident_frames == len(frames)
    out_res = _run(otfs, res, y)
    _cg_check(out_res, frames, ops, y, NMSE_TOL, "resident")
    say("cg small frames without LDS")
    mem = otfs.Plan([f.spec for f in frames], flags=otfs.NO_LDS_RESIDENT)
    assert mem.info().resident_frames == 0 and mem.info().lds_bytes == 0
    out_mem = _run(otfs, mem, y)
    _cg_check(out_mem, frames, ops, y, NMSE_TOL, "memory")
    assert np.array_equal(out_res[2]["iters"], out_mem[2]["iters"])
    for a, b in zip(split(out_res[0], frames), split(out_mem[0], frames)):
        assert O.nmse(a, b) <= 1e-10


@pytest.mark.parametrize("tile_elems,agent", [(256, 0), (128, 0), (640, 0), (256, 1)])
def test_cg_wide_doppler_neighbour_waits(otfs, tile_elems, agent):
    # Between the direction, H and H^H passes a tile waits only for the tiles owning the
    # rows it gathers (its band shifted by the Doppler range).  Wide and one-sided Doppler
    # ranges make those tile ranges wrap around the frame, cover most of it, or all of it.
    rng = np.random.default_rng(31 + tile_elems + agent)
    frames = [W.small_frame(rng, 64, 64, 6, (0, 20), (-20, 20), qam=16, snr_db=25.0,
                            max_iters=40),
              W.small_frame(rng, 64, 64, 5, (0, 9), (5, 30), qam=4, snr_db=20.0, max_iters=40),
              W.small_frame(rng, 128, 48, 7, (-10, 10), (-30, -3), qam=16, snr_db=22.0,
                            max_iters=40),
              W.small_frame(rng, 64, 40, 4, (0, 5), (-39, 39), qam=4, snr_db=15.0,
                            max_iters=40)]
    ops, xs, y = oracle_batch(frames)
    say("cg wide doppler", "tile_elems", tile_elems, "agent" if agent else "xcd",
        [(f.spec.M, f.spec.N, f.spec.P) for f in frames])
    plan = otfs.Plan([f.spec for f in frames], max_iters=40, rel_tol=1e-6,
                     tile_elems=tile_elems, flags=otfs.AGENT_BARRIER if agent else 0)
    _cg_check(_run(otfs, plan, y), frames, ops, y, NMSE_TOL)


@pytest.mark.parametrize("tile_elems", [0, 700, 200])
def test_cg_direction_in_gathers_identical_to_split(otfs, tile_elems):
    # Batches whose frames all have P <= 8 form p' = c + beta p inside the H pass's gathers;
    # the separate direction pass computes the same values in the same order, so the two
    # forms agree bit for bit (and both with the oracle).
    frames = _mixed_frames(41 + tile_elems, 7, [(128, 32), (64, 16), (100, 30), (256, 16)],
                           (1, 8), 12, 6)
    ops, xs, y = oracle_batch(frames)
    say("cg direction in gathers", "tile_elems", tile_elems,
        [(f.spec.M, f.spec.N, f.spec.P) for f in frames])
    fd = otfs.Plan([f.spec for f in frames], tile_elems=tile_elems, flags=otfs.NO_LDS_RESIDENT)
    sp = otfs.Plan([f.spec for f in frames], tile_elems=tile_elems,
                   flags=otfs.NO_LDS_RESIDENT | otfs.SPLIT_DIRECTION)
    assert fd.info().fused_direction_frames == len(frames)
    assert sp.info().fused_direction_frames == 0
    out_fd = _run(otfs, fd, y)
    out_sp = _run(otfs, sp, y)
    _cg_check(out_fd, frames, ops, y, NMSE_TOL, "direction in gathers")
    assert np.array_equal(out_fd[0], out_sp[0])
    assert np.array_equal(out_fd[1], out_sp[1])
    assert np.array_equal(out_fd[2]["iters"], out_sp[2]["iters"])
    # one frame with more paths sends the whole batch to the split form
    more = frames + _mixed_frames(43, 1, [(64, 16)], (9, 9), 12, 6)
    assert otfs.Plan([f.spec for f in more], tile_elems=tile_elems,
                     flags=otfs.NO_LDS_RESIDENT).info().fused_direction_frames == 0


def test_cg_fresh_plans_reusing_memory(otfs):
    # Regression: each new plan gets memory that earlier plans (other frame-to-XCD
    # assignments) used; stale cache lines must not leak into the solve.
    frames = _mixed_frames(11, 9, [(128, 32), (64, 16), (100, 30), (96, 8), (256, 16)],
                           (1, 9), 12, 4)
    ops, xs, y = oracle_batch(frames)
    for rep, te in enumerate([700, 350, 200, 700, 1024, 200]):
        say("cg fresh plan", rep, "tile_elems", te)
        plan = otfs.Plan([f.spec for f in frames], tile_elems=te)
        _cg_check(_run(otfs, plan, y), frames, ops, y, NMSE_TOL)
        del plan


def test_cg_plain_matches_oracle_and_fused(otfs):
    frames = _mixed_frames(12, 4, [(128, 32), (64, 16)], (2, 8), 8, 4)
    ops, xs, y = oracle_batch(frames)
    say("cg plain vs fused")
    plan = otfs.Plan([f.spec for f in frames], tile_elems=1024)
    xf, sf, stf = _run(otfs, plan, y, "fused")
    xp, sp_, stp = _run(otfs, plan, y, "plain")
    _cg_check((xp, sp_, stp), frames, ops, y, NMSE_TOL, "plain")
    assert np.all(np.abs(stf["iters"] - stp["iters"]) <= 1)
    # same algorithm and stop rule; the two forms may sum the per-thread partials of the
    # inner products in different orders (the staged fused form walks the band in blocks),
    # so they agree to FP32 rounding rather than bit for bit
    for a, b in zip(split(xf, frames), split(xp, frames)):
        assert O.nmse(a, b) <= 1e-6


def test_cg_fixed_iterations_and_first_step(otfs):
    frames = _mixed_frames(13, 3, [(64, 16), (128, 32)], (3, 6), 8, 4, max_iters=1, tol=0.0)
    ops, xs, y = oracle_batch(frames)
    say("cg one iteration")
    plan = otfs.Plan([f.spec for f in frames], max_iters=1, rel_tol=0.0)
    x, sym, st = _run(otfs, plan, y)
    assert np.all(st["iters"] == 1) and np.all(st["status"] == O_CAP)
    for i, (fr, xg) in enumerate(zip(frames, split(x, frames))):
        xr, _, _ = O.cg_lmmse(split(y, frames)[i], ops[i], fr.spec.lam, 1, 0.0)
        assert O.nmse(xg, xr) <= 1e-10
    frames10 = _mixed_frames(14, 3, [(64, 16)], (3, 6), 8, 4, max_iters=10, tol=0.0)
    ops, xs, y = oracle_batch(frames10)
    plan = otfs.Plan([f.spec for f in frames10], max_iters=10, rel_tol=0.0)
    x, sym, st = _run(otfs, plan, y)
    assert np.all(st["iters"] == 10)
    _cg_check((x, sym, st), frames10, ops, y, NMSE_TOL)


def test_cg_single_path_closed_form(otfs):
    rng = np.random.default_rng(15)
    M, N, h, lam = 64, 16, 0.6 + 0.9j, 0.05
    s = SpecLike(M, N, [3], [-2], [h], lam=lam, qam=4)
    y = _rand_c(rng, M * N)
    say("cg P=1")
    plan = otfs.Plan([s], max_iters=10, rel_tol=1e-5)
    x, sym, st = _run(otfs, plan, y)
    op = O.TwistedConvChannel(M, N, [h], [3], [-2])
    ref = op.apply_adjoint(y.astype(np.complex128)) / (abs(h) ** 2 + lam)
    assert st["iters"][0] == 1 and st["status"][0] == O_CONV
    assert O.nmse(x, ref) <= 1e-12


def test_cg_zero_and_nonfinite_frames_are_isolated(otfs):
    frames = _mixed_frames(16, 4, [(128, 32), (64, 16)], (3, 6), 8, 4)
    ops, xs, y = oracle_batch(frames)
    offs = np.concatenate([[0], np.cumsum([f.spec.E for f in frames])])
    say("cg isolation baseline")
    plan = otfs.Plan([f.spec for f in frames], tile_elems=1024)
    x0, s0, st0 = _run(otfs, plan, y)
    y2 = y.copy()
    y2[offs[1]:offs[2]] = 0                    # frame 1: H^H y = 0
    y2[offs[2] + 17] = np.nan                  # frame 2: a NaN sample
    say("cg isolation zero/nan")
    x2, s2, st2 = _run(otfs, plan, y2)
    assert st2["status"][1] == O_CONV and st2["iters"][1] == 0
    assert not np.any(x2[offs[1]:offs[2]])
    assert st2["status"][2] == 3               # OTFS_FRAME_NONFINITE
    for f in (0, 3):                           # untouched frames: bit-identical
        sl = slice(offs[f], offs[f + 1])
        assert np.array_equal(x0[sl], x2[sl]) and np.array_equal(s0[sl], s2[sl])
        assert st0["iters"][f] == st2["iters"][f]


def test_graph_replay_is_bit_identical(otfs):
    import torch
    frames = _mixed_frames(17, 5, [(128, 32), (64, 16), (256, 16)], (2, 8), 8, 4)
    ops, xs, y = oracle_batch(frames)
    say("graph replay")
    direct = otfs.Plan([f.spec for f in frames], tile_elems=2048)
    xd, sd, std_ = _run(otfs, direct, y)
    g = otfs.Plan([f.spec for f in frames], tile_elems=2048, flags=otfs.USE_GRAPH)
    with pytest.raises(otfs.OtfsError):                # the NULL stream cannot be captured
        g.lmmse_cg(to_dev(y), stream=torch.cuda.default_stream())
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        yd = to_dev(y)
        sym = torch.zeros(g.total_elems, dtype=torch.uint8, device="cuda")
        stats = g.new_stats()
        x = torch.empty(g.total_elems, dtype=torch.complex64, device="cuda")
        for rep in range(4):
            x.fill_(float("nan"))
            sym.fill_(255)
            torch.zeros(1000, device="cuda").sum()      # unrelated eager work in between
            g.lmmse_cg(yd, x, sym, stats)
            side.synchronize()
            assert np.array_equal(x.cpu().numpy(), xd), rep
            assert np.array_equal(sym.cpu().numpy(), sd), rep
            assert np.array_equal(otfs.stats_numpy(stats)["iters"], std_["iters"])


def test_cg_fp64_refresh(otfs):
    frames = _mixed_frames(18, 3, [(128, 32), (256, 16)], (4, 12), 10, 4, qams=(64,),
                           snr=(30, 30))
    ops, xs, y = oracle_batch(frames)
    say("cg refresh every 5")
    plan = otfs.Plan([f.spec for f in frames], refresh_every=5, tile_elems=1024)
    _cg_check(_run(otfs, plan, y), frames, ops, y, NMSE_TOL)


def test_cg_bf16_stored_mode(otfs):
    import torch
    frames = _mixed_frames(19, 3, [(128, 32), (256, 16)], (4, 12), 10, 4, qams=(64,),
                           snr=(30, 30))
    ops, xs, y = oracle_batch(frames)
    yb = torch.view_as_real(to_dev(y)).to(torch.bfloat16).contiguous().view(-1)
    y_rounded = torch.view_as_complex(yb.view(-1, 2).float()).cpu().numpy()
    say("cg bf16 y + stored D")
    plan = otfs.Plan([f.spec for f in frames], refresh_every=10,
                     flags=otfs.Y_BF16 | otfs.D_STORED_BF16, tile_elems=1024)
    sym = torch.zeros(plan.total_elems, dtype=torch.uint8, device="cuda")
    stats = plan.new_stats()
    x = plan.lmmse_cg(yb, sym=sym, stats=stats).cpu().numpy()
    st = otfs.stats_numpy(stats)
    for i, (fr, xg) in enumerate(zip(frames, split(x, frames))):
        xr, _, _ = O.cg_lmmse(split(y_rounded, frames)[i], ops[i], fr.spec.lam,
                              fr.spec.max_iters, fr.spec.tol)
        assert O.nmse(xg, xr) <= NMSE_TOL_BF16, i
        assert st["status"][i] in (O_CONV, O_CAP)


def test_wait_limit_gives_up_cleanly(otfs):
    # The host shortens the bound of the kernel's own waits to nothing: waits that are not
    # satisfied at once give up, the launch-wide abort word ends every other wait, the
    # affected frames report OTFS_FRAME_TIMEOUT and every workgroup exits normally.  The
    # same plan with the default bound then solves the batch correctly.
    import torch
    frames = _mixed_frames(51, 12, [(256, 64), (128, 32), (512, 16)], (3, 8), 12, 4)
    ops, xs, y = oracle_batch(frames)
    plan = otfs.Plan([f.spec for f in frames], tile_elems=1024, flags=otfs.NO_LDS_RESIDENT)
    assert plan.info().grid > len(frames)
    say("wait limit 0")
    plan.set_wait_limit(0)
    x, sym, st = _run(otfs, plan, y)
    say("  statuses", list(st["status"]))
    assert np.all(np.isin(st["status"], [O_CONV, O_CAP, 5]))
    assert np.count_nonzero(st["status"] == 5) >= 1
    say("default wait limit again")
    plan.set_wait_limit(-1)
    _cg_check(_run(otfs, plan, y), frames, ops, y, NMSE_TOL)


def test_cg_stored_c64_table(otfs):
    # the SS table of Eq. ds_repr kept in complex64: same results as the on-the-fly
    # coefficients up to the rounding of the wrap factors, on every wrap case
    rng = np.random.default_rng(61)
    specs = _edge_specs(rng)
    say("stored c64 apply parity", [(s.M, s.N, s.P) for s in specs])
    plan = otfs.Plan(specs, flags=otfs.D_STORED_C64)
    E = plan.total_elems
    x = _rand_c(rng, E)
    y = _rand_c(rng, E)
    yh = plan.apply_H(to_dev(x)).cpu().numpy()
    xh = plan.apply_HH(to_dev(y)).cpu().numpy()
    o = 0
    for s in specs:
        op = O.TwistedConvChannel(s.M, s.N, s.h, s.tau, s.nu)
        sl = slice(o, o + s.E)
        scale = np.abs(s.h).sum()
        assert np.abs(yh[sl] - op.apply(x[sl].astype(np.complex128))).max() <= \
            1e-5 * scale * np.abs(x[sl]).max(), (s.M, s.N)
        assert np.abs(xh[sl] - op.apply_adjoint(y[sl].astype(np.complex128))).max() <= \
            1e-5 * scale * np.abs(y[sl]).max(), (s.M, s.N)
        o += s.E
    frames = _mixed_frames(62, 6, [(128, 32), (64, 16), (256, 16)], (2, 12), 10, 4)
    ops, xs, yy = oracle_batch(frames)
    say("cg stored c64 table, refresh every 10")
    plan = otfs.Plan([f.spec for f in frames], refresh_every=10, tile_elems=1024,
                     flags=otfs.D_STORED_C64)
    _cg_check(_run(otfs, plan, yy), frames, ops, yy, NMSE_TOL)
