"""Full-size GPU parity of the workload batches against the FP64 oracle, every frame.

Each batch is solved on the GPU at its real size, in the launch configuration the
benchmark times, and every frame is compared with the oracle's CG under the identical
stop rule (Algorithm 1 with the relative-residual stop), on the same received y: the
oracle makes y (complex128, rounded once to complex64) in a pool of worker processes
that run NumPy only.  Per frame: NMSE of the estimate, the iteration count, and the hard
decisions (Eq. demod) -- equal to the oracle's except where the oracle's estimate is
closer to a decision boundary than the GPU's estimate is to it (helpers.check_decisions);
the number of such differing decisions is printed.

The 128 x (1024, 256) batch runs in four modes: complex64 with the FP64 true-residual
refresh every 10 iterations, the same with the SS table of Eq. ds_repr stored in
complex64, and y plus the stored table in bf16 (stated separately: NMSE <= 1e-4 against
the oracle run on the bf16-rounded y, with the symbol-error rates beside it).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import (bf16_round, check_decisions, iters_close, oracle_received, oracle_solve,
                     pool_map, say, ser, split, to_dev)

pytestmark = pytest.mark.gpu

NMSE_TOL = 1e-5          # FP32 path vs FP64 oracle, per frame
NMSE_TOL_BF16 = 1e-4     # y and D stored as bf16
O_CONV, O_CAP = 1, 2


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _gpu_solve(otfs, specs, y, y_dev=None, **plan_kw):
    import torch
    plan = otfs.Plan(specs, max_iters=specs[0].max_iters, rel_tol=specs[0].tol, **plan_kw)
    yd = to_dev(y) if y_dev is None else y_dev
    sym = torch.zeros(plan.total_elems, dtype=torch.uint8, device="cuda")
    stats = plan.new_stats()
    x = plan.lmmse_cg(yd, sym=sym, stats=stats)
    torch.cuda.synchronize()
    out = x.cpu().numpy(), sym.cpu().numpy(), otfs.stats_numpy(stats)
    del plan, x, sym, stats, yd
    torch.cuda.empty_cache()
    return out


def _compare(name, frames, gpu, refs, tol, ys=None, check_iters=True):
    """Every frame: NMSE, iterations, decisions.  refs[i] = (y, x_ref, iters, rel)."""
    xg, symg, st = gpu
    xs, syms = split(xg, frames), split(symg, frames)
    nm = np.zeros(len(frames))
    diffs = ser_gpu = ser_ref = 0.0
    n_sym = 0
    for i, fr in enumerate(frames):
        sp = fr.spec
        _, xr, it_r, rel_r = refs[i]
        nm[i] = O.nmse(xs[i], xr)
        assert nm[i] <= tol, f"{name} frame {i} ({sp.M}x{sp.N}, P={sp.P}): NMSE {nm[i]:.3e}"
        assert st["status"][i] in (O_CONV, O_CAP), (name, i, st["status"][i])
        if check_iters:
            capped = rel_r > sp.tol * 1.5 and it_r == sp.max_iters
            assert iters_close(int(st["iters"][i]), it_r, capped), (name, i, st["iters"][i], it_r)
        diffs += check_decisions(syms[i], xs[i], xr, sp.qam)
        ser_gpu += ser(syms[i], fr.sym) * sp.E
        ser_ref += ser(O.qam_decide(xr, sp.qam), fr.sym) * sp.E
        n_sym += sp.E
    say(name, f"frames {len(frames)}: NMSE worst {nm.max():.3e} mean {nm.mean():.3e}; "
              f"decisions differing from the oracle {int(diffs)} of {n_sym}; "
              f"SER gpu {ser_gpu / n_sym:.4e} oracle {ser_ref / n_sym:.4e}; "
              f"iterations {int(st['iters'].min())}..{int(st['iters'].max())}")
    return nm


def _all_frames(oracle_pool, name):
    frames = list(W.iter_frames(name))
    say("full size", name, len(frames), "frames: oracle CG of every frame")
    refs = pool_map(oracle_pool, oracle_solve, [(f, None) for f in frames], name)
    y = np.concatenate([r[0] for r in refs]).astype(np.complex64)
    return frames, refs, y


def test_fullsize_batch64_512x128_every_frame(otfs, oracle_pool):
    frames, refs, y = _all_frames(oracle_pool, "batch64_512x128")
    say("gpu solve batch64_512x128")
    gpu = _gpu_solve(otfs, [f.spec for f in frames], y)
    _compare("batch64_512x128", frames, gpu, refs, NMSE_TOL)


def test_fullsize_uneven256_every_frame(otfs, oracle_pool):
    frames, refs, y = _all_frames(oracle_pool, "uneven256")
    say("gpu solve uneven256")
    gpu = _gpu_solve(otfs, [f.spec for f in frames], y)
    _compare("uneven256", frames, gpu, refs, NMSE_TOL)


# ---- 128 x (1024, 256), P = 16, 64-QAM, 30 dB -------------------------------------------
C5 = "batch128_1024x256"
C5_REFRESH = 10
C5_BF16_SAMPLE = list(range(0, 128, 8))      # 16 frames spread over the batch


@pytest.fixture(scope="module")
def c5(oracle_pool):
    frames, refs, y = _all_frames(oracle_pool, C5)
    return {"frames": frames, "refs": refs, "y": y, "c64": None}


def test_fullsize_batch128_1024x256_c64_refresh(otfs, c5):
    say("gpu solve", C5, "complex64, FP64 refresh every", C5_REFRESH)
    frames = c5["frames"]
    gpu = _gpu_solve(otfs, [f.spec for f in frames], c5["y"], refresh_every=C5_REFRESH)
    c5["c64"] = gpu
    _compare(C5 + " c64 refresh", frames, gpu, c5["refs"], NMSE_TOL)


def test_fullsize_batch128_1024x256_stored_c64_refresh(otfs, c5):
    say("gpu solve", C5, "stored complex64 D, FP64 refresh every", C5_REFRESH)
    frames = c5["frames"]
    gpu = _gpu_solve(otfs, [f.spec for f in frames], c5["y"], refresh_every=C5_REFRESH,
                     flags=otfs.D_STORED_C64)
    _compare(C5 + " stored-c64 refresh", frames, gpu, c5["refs"], NMSE_TOL)


def test_fullsize_batch128_1024x256_bf16_refresh(otfs, c5, oracle_pool):
    import torch
    frames = c5["frames"]
    bits, y_rounded = bf16_round(c5["y"])
    sample = C5_BF16_SAMPLE
    say(C5, "bf16: oracle CG on the bf16-rounded y of", len(sample), "frames")
    ys = split(y_rounded, frames)
    refs = pool_map(oracle_pool, oracle_solve, [(frames[i], ys[i]) for i in sample], "bf16")
    say("gpu solve", C5, "bf16 y and stored bf16 D, FP64 refresh every", C5_REFRESH)
    yb = torch.from_numpy(bits.view(np.int16)).to("cuda").view(torch.bfloat16)
    xg, symg, st = _gpu_solve(otfs, [f.spec for f in frames], None, y_dev=yb,
                              refresh_every=C5_REFRESH, flags=otfs.Y_BF16 | otfs.D_STORED_BF16)
    xs, syms = split(xg, frames), split(symg, frames)
    sub = [frames[i] for i in sample]
    gpu_sub = (np.concatenate([xs[i] for i in sample]), np.concatenate([syms[i] for i in sample]),
               st[sample])
    nm = _compare(C5 + " bf16 vs oracle(bf16 y)", sub, gpu_sub, refs, NMSE_TOL_BF16)
    # against the complex64 GPU solve and the oracle on the unrounded y
    if c5["c64"] is not None:
        xc, symc, _ = c5["c64"]
        xcs, symcs = split(xc, frames), split(symc, frames)
        nm64 = [O.nmse(xs[i], xcs[i]) for i in sample]
        flips = sum(int(np.count_nonzero(syms[i] != symcs[i])) for i in sample)
        n = sum(frames[i].spec.E for i in sample)
        ser_b = np.mean([ser(syms[i], frames[i].sym) for i in sample])
        ser_c = np.mean([ser(symcs[i], frames[i].sym) for i in sample])
        say(C5, f"bf16 vs complex64 GPU: NMSE worst {max(nm64):.3e}; decisions differing "
                f"{flips} of {n}; SER bf16 {ser_b:.4e} complex64 {ser_c:.4e} "
                f"(delta {ser_b - ser_c:+.2e})")
    nm_exact = [O.nmse(xs[i], c5["refs"][i][1]) for i in sample]
    say(C5, f"bf16 vs oracle on the unrounded y: NMSE worst {max(nm_exact):.3e}")
    assert max(nm) <= NMSE_TOL_BF16
