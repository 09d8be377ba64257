"""The whole receiver on the device for the fractional delay-Doppler workload (Veh-A
profile of Sec. V, Doppler nu_max cos(2 pi U)): time-domain pilot and data frames through
the fractional channel (made by the oracle), then on the GPU the DZT (MFMA), the path table
from the pilot (Y . E_twist, threshold 0.08 as in Sec. V, and 0.03 from the operating range
of Sec. VI), LMMSE-CG with Algorithm 1's fixed 10 iterations, decisions and bit errors
(receiver.receive).  Against the FP64 oracle chain:
the DZT element by element, the selected bins (equal except where a bin's magnitude lies
within the FP32 error of the threshold), the equaliser (the oracle's CG run with the
device's path table, NMSE <= 1e-5), decisions, and the bit-error counts.  With fractional
delays and Dopplers the structured-sparse channel is an approximation (Sec. IV-B); the BER
printed here is that of the approximation."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import check_decisions, say, to_dev

pytestmark = pytest.mark.gpu
CAP, ITERS = 64, 10


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("snr_db,qam,theta", [(10.0, 4, 0.08), (20.0, 4, 0.08), (30.0, 4, 0.08),
                                              (10.0, 16, 0.08), (20.0, 16, 0.08), (30.0, 16, 0.08),
                                              (30.0, 4, 0.03), (30.0, 16, 0.03)])
def test_fractional_receiver_chain_matches_oracle(otfs, snr_db, qam, theta):
    import torch

    from paper_2604_02266_amd import receiver
    M, N, npk, nd = 128, 32, 3, 2
    rng = np.random.default_rng(int(snr_db) * 10 + qam)
    packets = [W.veh_a_packet(rng, M, N, ndata=nd, qam=qam, snr_db=snr_db) for _ in range(npk)]
    rec = [O.veh_a_received(pk) for pk in packets]
    yp = np.concatenate([r[0] for r in rec])
    ys = np.concatenate([r[1].reshape(-1) for r in rec])
    tx = np.concatenate([pk.sym.reshape(-1) for pk in packets]).astype(np.uint8)
    lam = packets[0].lam
    say("receiver chain", M, N, "snr", snr_db, "qam", qam)
    out = receiver.receive(to_dev(yp), to_dev(ys), M, N, lam, qam, theta=theta, capacity=CAP,
                           max_iters=ITERS, rel_tol=0.0, sym_tx=torch.from_numpy(tx).cuda())
    torch.cuda.synchronize()
    pilot_dd = out["pilot_dd"].cpu().numpy()
    y_dd = out["y_dd"].cpu().numpy()
    xg = out["xhat"].cpu().numpy()
    sym = out["sym"].cpu().numpy()
    errs = out["errs"].cpu().numpy()
    npaths = out["npaths"].cpu().numpy()
    E = M * N
    tol = 2e-6 * math.sqrt(N)
    near_total = 0
    ber_g = ber_o = 0
    bits = 2 * int(round(math.log2(math.sqrt(qam))))
    for p, pk in enumerate(packets):
        Yp = O.dzt(yp[p * E:(p + 1) * E].astype(np.complex128), M, N)
        assert np.abs(pilot_dd[p * E:(p + 1) * E] - Yp).max() <= tol * np.abs(Yp).max()
        est = O.pilot_estimate_hadamard(Yp, M, N)
        t_o, v_o, g_o = O.threshold_paths(est, theta, np.float32)
        tg, vg, gg = out["plan"].get_paths(p * nd)
        assert int(npaths[p]) >= tg.size
        so = {(int(a), int(b)) for a, b in zip(t_o[:CAP], v_o[:CAP])}
        sg = {(int(a), int(b)) for a, b in zip(tg, vg)}
        K0, L0 = M // 2, N // 2
        for (t, v) in so ^ sg:     # a differing bin must sit at the threshold
            assert abs(abs(est[t + K0, v + L0]) - theta) <= 1e-5, (t, v, abs(est[t + K0, v + L0]))
            near_total += 1
        op_g = O.TwistedConvChannel(M, N, gg.astype(np.complex128), tg, vg)
        for d in range(nd):
            f = p * nd + d
            sl = slice(f * E, (f + 1) * E)
            ydd = O.dzt(ys[sl].astype(np.complex128), M, N)
            assert np.abs(y_dd[sl] - ydd).max() <= tol * np.abs(ydd).max()
            xr, _, _ = O.cg_lmmse(ydd, op_g, lam, ITERS, 0.0)
            assert O.nmse(xg[sl], xr) <= 1e-5, (f, O.nmse(xg[sl], xr))
            check_decisions(sym[sl], xg[sl], xr, qam)
            assert int(errs[f]) == O.bit_errors(sym[sl], pk.sym[d], qam)
            # the oracle's own chain (its DZT, its threshold set)
            op_o = O.TwistedConvChannel(M, N, g_o[:CAP], t_o[:CAP], v_o[:CAP])
            xo, _, _ = O.cg_lmmse(ydd, op_o, lam, ITERS, 0.0)
            ber_o += O.bit_errors(O.qam_decide(xo, qam), pk.sym[d], qam)
            ber_g += int(errs[f])
    nbits = npk * nd * E * bits
    say(f"fractional Veh-A, {snr_db} dB, {qam}-QAM, theta {theta}: paths above theta {list(npaths)}; "
        f"bins differing at the threshold {near_total}; BER gpu {ber_g / nbits:.4e} "
        f"oracle chain {ber_o / nbits:.4e}")
