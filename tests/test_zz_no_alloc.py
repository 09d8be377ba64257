"""The entry point that allocates nothing (otfs_lmmse_cg_noalloc), through the C ABI: it
binds the plan to the library's static per-device scratch and must give the same results,
bit for bit, as otfs_lmmse_cg on a caller-allocated workspace, on two calls in a row (the
second with a smaller batch, so the scratch holds stale state from the first), and reject
a plan whose workspace exceeds the scratch."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import oracle_batch, say, split, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _frames(seed, shapes):
    rng = np.random.default_rng(seed)
    return [W.small_frame(rng, M, N, int(rng.integers(2, 9)), (0, min(12, M - 1)),
                          (-min(4, N - 1), min(4, N - 1)), qam=16, snr_db=22.0, max_iters=40,
                          tol=1e-6) for (M, N) in shapes]


def _solve(otfs, plan, y, noalloc):
    import torch
    sym = torch.zeros(plan.total_elems, dtype=torch.uint8, device="cuda")
    stats = plan.new_stats()
    fn = plan.lmmse_cg_noalloc if noalloc else plan.lmmse_cg
    x = fn(to_dev(y), sym=sym, stats=stats)
    torch.cuda.synchronize()
    return x.cpu().numpy(), sym.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("refresh", [0, 7])
def test_noalloc_equals_workspace_entry_point(otfs, refresh):
    big = _frames(81, [(256, 64), (128, 32), (512, 16), (64, 16), (128, 64), (37, 11)])
    small = _frames(82, [(128, 32), (64, 16)])
    for name, frames in (("first call", big), ("second call, smaller", small)):
        ops, _, y = oracle_batch(frames)
        say("noalloc", name, [(f.spec.M, f.spec.N, f.spec.P) for f in frames], "refresh", refresh)
        plan = otfs.Plan([f.spec for f in frames], max_iters=40, rel_tol=1e-6,
                         refresh_every=refresh)
        ws, _ = plan.workspace_bytes()
        assert ws <= 64 << 20
        ref = _solve(otfs, plan, y, noalloc=False)
        got = _solve(otfs, plan, y, noalloc=True)
        assert np.array_equal(ref[0].view(np.uint32), got[0].view(np.uint32)), name
        assert np.array_equal(ref[1], got[1]), name
        assert np.array_equal(ref[2], got[2]), name
        # and the oracle's bar on one frame of each call
        xr, _, _ = O.cg_lmmse(split(y, frames)[0], ops[0], frames[0].spec.lam, 40, 1e-6)
        assert O.nmse(split(got[0], frames)[0], xr) <= 1e-5


def test_noalloc_rejects_a_plan_beyond_the_scratch(otfs):
    import torch
    rng = np.random.default_rng(83)
    specs = [W.small_frame(rng, 512, 512, 4, (0, 8), (-4, 4)).spec for _ in range(8)]
    plan = otfs.Plan(specs, bind=False)
    ws, E = plan.workspace_bytes()
    assert ws > 64 << 20
    y = torch.zeros(E, dtype=torch.complex64, device="cuda")
    with pytest.raises(otfs.OtfsError) as ei:
        plan.lmmse_cg_noalloc(y)
    assert ei.value.status == otfs.E_NOMEM
