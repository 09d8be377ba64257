"""GPU parity of the bit-error measurement and the per-iteration CG trace behind the
BER-driven iteration budget (Sec. IV-C, Eq. ber_convergence) against the FP64 oracle.

The GPU runs the fused solve one iteration per launch and records, after each iteration,
the bit errors (Gray map per axis) of its current decisions; the oracle runs its CG with
the same fixed count and demaps its own decisions (taken in FP32 on its estimate rounded
to complex64).  Per iteration the two counts may differ only by decisions whose oracle
estimate lies within 1e-3 of a decision boundary; the convergence iteration of the BER
curves must agree."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import check_decisions, oracle_batch, say, split, to_dev

pytestmark = pytest.mark.gpu
ITERS = 16


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _frames(seed, shapes, qams, snrs):
    rng = np.random.default_rng(seed)
    out = []
    for i, (M, N) in enumerate(shapes):
        out.append(W.small_frame(rng, M, N, int(rng.integers(3, 9)), (0, min(16, M - 1)),
                                 (-min(4, N - 1), min(4, N - 1)), qam=qams[i % len(qams)],
                                 snr_db=snrs[i % len(snrs)], max_iters=ITERS, tol=0.0))
    return out


@pytest.mark.parametrize("refresh", [0, 5])
def test_trace_bit_errors_match_oracle(otfs, refresh):
    import torch
    frames = _frames(41, [(128, 32), (64, 16), (256, 16), (96, 24)], (4, 16, 64), (8.0, 18.0, 30.0))
    ops, xs, y = oracle_batch(frames)
    say("cg trace", [(f.spec.M, f.spec.N, f.spec.P, f.spec.qam) for f in frames], "refresh", refresh)
    plan = otfs.Plan([f.spec for f in frames], max_iters=ITERS, rel_tol=0.0,
                     refresh_every=refresh)
    tx = torch.from_numpy(np.concatenate([f.sym for f in frames]).astype(np.uint8)).cuda()
    stats = plan.new_stats()
    xg, sym, errs = plan.lmmse_cg_trace(to_dev(y), tx, stats=stats)
    torch.cuda.synchronize()
    errs = errs.cpu().numpy()
    xg, sym = xg.cpu().numpy(), sym.cpu().numpy()
    # the final results equal the plain fused solve's and the oracle's
    x2 = plan.lmmse_cg(to_dev(y)).cpu().numpy()
    assert np.array_equal(x2.view(np.uint32), xg.view(np.uint32))
    ys = split(y, frames)
    for i, fr in enumerate(frames):
        sp = fr.spec
        tr = O.cg_lmmse_trace(ys[i], ops[i], sp.lam, ITERS)
        bits = 2 * int(round(np.log2(np.sqrt(sp.qam))))
        ber_o, ber_g = [], []
        for k in range(ITERS):
            xr = tr[k]
            dr = O.qam_decide(xr.astype(np.complex64), sp.qam, np.float32)
            eo = O.bit_errors(dr, fr.sym, sp.qam)
            near = int(np.count_nonzero(O.decision_margin(xr, sp.qam) < 1e-3))
            assert abs(int(errs[k, i]) - eo) <= near * bits, (i, k, int(errs[k, i]), eo, near)
            ber_o.append(eo / (sp.E * bits))
            ber_g.append(int(errs[k, i]) / (sp.E * bits))
        # the last row counts the final decisions exactly
        assert int(errs[ITERS - 1, i]) == O.bit_errors(split(sym, frames)[i], fr.sym, sp.qam)
        check_decisions(split(sym, frames)[i], split(xg, frames)[i], tr[-1], sp.qam)
        kg, ko = O.ber_convergence(ber_g), O.ber_convergence(ber_o)
        say(f"frame {i}: BER after 1/{ITERS} it {ber_g[0]:.3e}/{ber_g[-1]:.3e}; "
            f"converged at {kg} (oracle {ko})")
        assert kg == ko
    # the stand-alone count of the final decisions
    e2 = plan.bit_errors(torch.from_numpy(sym).cuda(), tx).cpu().numpy()
    assert np.array_equal(e2, errs[ITERS - 1])
