"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each pin is independent of the code under test: values printed in the paper (fixtures in
tests/golden/ with their citation), the three other constructions of the channel matrix
(Eq. Hdd as printed, the shift-operator product, the DZT-conjugated time-domain channel),
closed forms (P=1 CG, noiseless recovery, unitarity), a textbook routine (Cholesky via
LAPACK) and brute force (Eq. demod over the whole constellation).  The mutation tests at
the end plant plausible mistakes in a copy of the operator and check that the pins catch
them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

RNG = np.random.default_rng(20260402)


def _rand_c(n, rng=RNG):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


# shapes and paths covering every wrap case: tau at 0 and M-1, negative tau, nu at
# +-(N-1), M or N equal to one, sizes that are not powers of two, repeated bins mod (M,N)
OPERATOR_CASES = [
    (8, 4, [0, 7, -3, 2, 1, 0], [0, 3, -2, -3, 1, 2]),
    (5, 3, [4, -4, 2], [2, -2, 1]),
    (1, 4, [0, 0], [3, -3]),
    (6, 1, [5, -5, 2], [0, 0, 0]),
    (7, 5, [6, -6, 0, 3], [-4, 4, 0, -1]),
    (4, 4, [1, -3], [2, -2]),            # tau=-3 and tau=1 hit the same column set
    (12, 2, [11, 0, -11], [1, -1, 0]),
]


@pytest.mark.parametrize("M,N,tau,nu", OPERATOR_CASES)
def test_four_constructions_agree(M, N, tau, nu):
    h = _rand_c(len(tau))
    op = O.TwistedConvChannel(M, N, h, tau, nu)
    Hdef = O.dense_from_operator(op)
    Heq = O.dense_H_eq_Hdd(M, N, h, tau, nu)
    Hsh = O.dense_H_shift_ops(M, N, h, tau, nu)
    Htd = O.dense_H_timedomain(M, N, h, tau, nu)
    scale = np.abs(h).sum()
    assert np.abs(Hdef - Heq).max() <= 1e-13 * scale
    assert np.abs(Hdef - Hsh).max() <= 1e-13 * scale
    assert np.abs(Hdef - Htd).max() <= 1e-13 * scale


@pytest.mark.parametrize("M,N,tau,nu", OPERATOR_CASES)
def test_adjoint_is_conjugate_transpose(M, N, tau, nu):
    h = _rand_c(len(tau))
    op = O.TwistedConvChannel(M, N, h, tau, nu)
    H = O.dense_H_eq_Hdd(M, N, h, tau, nu)
    y = _rand_c(M * N)
    assert np.abs(op.apply_adjoint(y) - H.conj().T @ y).max() <= 1e-12
    x = _rand_c(M * N)
    lhs = np.vdot(op.apply(x), y)
    rhs = np.vdot(x, op.apply_adjoint(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_worked_example_8x2(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "worked_example_8x2.json")))
    M, N = g["M"], g["N"]
    K0, L0 = g["pilot"]
    tau = [kp - K0 for kp, lp in g["paths_pilot_grid"]]
    nu = [lp - L0 for kp, lp in g["paths_pilot_grid"]]
    op = O.TwistedConvChannel(M, N, [1.0, 0.7 - 0.2j], tau, nu)
    H = O.dense_from_operator(op)
    cols = np.nonzero(np.abs(H[g["row"]]) > 1e-12)[0].tolist()
    assert cols == g["row_columns"]
    assert H.size == g["dense_multiplications"]
    assert np.count_nonzero(np.abs(H) > 1e-12) == g["ss_multiplications"]


def test_ss_entry_count_48x32(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "ss_memory_48x32.json")))
    M, N, P = g["M"], g["N"], g["P"]
    rng = np.random.default_rng(5)
    fr = W.small_frame(rng, M, N, P, (-4, 4), (-3, 3))
    H = O.dense_H_eq_Hdd(M, N, fr.spec.h, fr.spec.tau, fr.spec.nu)
    nnz = int(np.count_nonzero(np.abs(H) > 1e-12))
    assert nnz == g["ss_entries"]
    assert round(H.size / 1e6, 1) == g["dense_entries_approx"] / 1e6
    assert round(H.size / nnz, 1) == g["reduction"]
    big = 8 * (g["big_M"] ** 2) * (g["big_N"] ** 2) / 1e9
    assert round(big, 1) == g["big_dense_GB"]


@pytest.mark.parametrize("M,N,tau,nu", [(8, 4, 3, -2), (5, 3, -4, 2), (16, 8, 15, 7)])
def test_single_path_is_scaled_unitary(M, N, tau, nu):
    h = 0.8 - 0.3j
    H = O.dense_H_eq_Hdd(M, N, [h], [tau], [nu])
    G = H.conj().T @ H
    assert np.abs(G - abs(h) ** 2 * np.eye(M * N)).max() <= 1e-13


def test_dzt_is_unitary_and_matches_direct_sums():
    M, N = 6, 4
    Z = O.dzt_matrix(M, N)
    assert np.abs(Z @ Z.conj().T - np.eye(M * N)).max() <= 1e-13
    x = _rand_c(M * N)
    assert np.abs(O.dzt(O.idzt(x, M, N), M, N) - x).max() <= 1e-12
    assert np.abs(Z @ x - O.dzt(x, M, N)).max() <= 1e-12
    assert np.abs(Z.conj().T @ x - O.idzt(x, M, N)).max() <= 1e-12


@pytest.mark.parametrize("M,N", [(16, 8), (32, 16), (64, 16)])
def test_pilot_impulse_response_recovers_paths(M, N):
    # non-wrapping paths (Eq. heff support): |tau| < M/2, |nu| < N/2
    rng = np.random.default_rng(M * 100 + N)
    fr = W.small_frame(rng, M, N, 5, (-(M // 2) + 1, M // 2 - 1), (-(N // 2) + 1, N // 2 - 1))
    sp = fr.spec
    op = O.TwistedConvChannel(M, N, sp.h, sp.tau, sp.nu)
    d = np.zeros((M, N), dtype=np.complex128)
    d[M // 2, N // 2] = 1.0
    yp = op.apply(O.vec(d))
    est = O.pilot_estimate_direct(yp, M, N)
    had = O.pilot_estimate_hadamard(yp, M, N)
    for t, v, hp in zip(sp.tau, sp.nu, sp.h):
        assert abs(est[(int(t), int(v))] - hp) <= 1e-14
        assert abs(had[t + M // 2, v + N // 2] - hp) <= 1e-14
    # every other bin is empty
    pathset = {(int(t), int(v)) for t, v in zip(sp.tau, sp.nu)}
    for key, val in est.items():
        if key not in pathset:
            assert abs(val) <= 1e-14


@pytest.mark.parametrize("M,N", [(16, 8), (32, 16)])
def test_threshold_selects_the_true_paths(M, N):
    # Eq. heff_thres on a noiseless pilot: with every |h_p| above theta and the paths inside
    # the estimate's support, the selected set is the channel's own path set, in vector
    # order, with the channel's gains; it also agrees with thresholding the direct form of
    # Eq. heff, and a larger theta selects a subset.
    rng = np.random.default_rng(M + 7 * N)
    fr = W.small_frame(rng, M, N, 6, (-(M // 2) + 1, M // 2 - 1), (-(N // 2) + 1, N // 2 - 1))
    sp = fr.spec
    h = sp.h / np.abs(sp.h) * (0.2 + rng.uniform(0, 1, sp.P))      # every |h_p| >= 0.2
    op = O.TwistedConvChannel(M, N, h, sp.tau, sp.nu)
    yp = op.apply(O.pilot_frame(M, N))
    tau, nu, g = O.threshold_paths(O.pilot_estimate_hadamard(yp, M, N), 0.08)
    order = np.argsort((np.asarray(sp.nu) + N // 2) * M + (np.asarray(sp.tau) + M // 2))
    assert np.array_equal(tau, np.asarray(sp.tau)[order])
    assert np.array_equal(nu, np.asarray(sp.nu)[order])
    assert np.abs(g - h[order]).max() <= 1e-14
    direct = O.pilot_estimate_direct(yp, M, N)
    sel = sorted(((v + N // 2) * M + (t + M // 2)) for (t, v), val in direct.items()
                 if abs(val) > 0.08)
    assert sel == sorted(((nu + N // 2) * M + (tau + M // 2)).tolist())
    t2, _, _ = O.threshold_paths(O.pilot_estimate_hadamard(yp, M, N), 0.5)
    assert set(t2.tolist()) <= set(tau.tolist())
    # noise well below theta selects nothing else
    w = 0.01 * (rng.standard_normal(M * N) + 1j * rng.standard_normal(M * N)) / math.sqrt(2)
    tau_n, nu_n, _ = O.threshold_paths(O.pilot_estimate_hadamard(yp + w, M, N), 0.08)
    assert np.array_equal(tau_n, tau) and np.array_equal(nu_n, nu)


def test_cg_single_path_closed_form():
    # P=1: H^H H = |h|^2 I, so one CG step lands on H^H y / (|h|^2 + lam)
    M, N = 16, 8
    h, lam = 0.6 + 0.9j, 0.05
    op = O.TwistedConvChannel(M, N, [h], [3], [-2])
    y = _rand_c(M * N)
    x, it, rel = O.cg_lmmse(y, op, lam, 10, 1e-12)
    assert it == 1
    ref = op.apply_adjoint(y) / (abs(h) ** 2 + lam)
    assert np.abs(x - ref).max() <= 1e-13


def test_cg_noiseless_exact_recovery():
    rng = np.random.default_rng(11)
    fr = W.small_frame(rng, 16, 8, 4, (0, 4), (-2, 2), qam=16)
    sp = fr.spec
    op = O.TwistedConvChannel(sp.M, sp.N, sp.h, sp.tau, sp.nu)
    x = O.qam_points(fr.sym, 16)
    x_hat, it, rel = O.cg_lmmse(op.apply(x), op, 0.0, sp.E, 1e-13)
    assert rel <= 1e-13
    assert np.abs(x_hat - x).max() <= 1e-9


@pytest.mark.parametrize("M,N,P,snr", [(8, 4, 3, 10.0), (16, 8, 5, 20.0), (12, 6, 4, 30.0)])
def test_cg_converges_to_dense_lmmse(M, N, P, snr):
    rng = np.random.default_rng(M * N * P)
    fr = W.small_frame(rng, M, N, P, (-(M - 1), M - 1), (-(N - 1), N - 1), snr_db=snr)
    sp = fr.spec
    op, x, y = O.received_frame(fr)
    H = O.dense_H_timedomain(M, N, sp.h, sp.tau, sp.nu)     # independent construction
    ref = O.lmmse_dense(y, H, sp.lam)
    got, it, rel = O.cg_lmmse(y, op, sp.lam, 4 * sp.E, 1e-13)
    assert rel <= 1e-13
    assert O.nmse(got, ref) <= 1e-22


def test_cg_fixed_count_and_first_step():
    rng = np.random.default_rng(3)
    fr = W.small_frame(rng, 8, 4, 3, (0, 3), (-1, 1))
    sp = fr.spec
    op, x, y = O.received_frame(fr)
    _, it, _ = O.cg_lmmse(y, op, sp.lam, 7, 0.0)
    assert it == 7
    # first CG iterate = steepest-descent step along b with exact line search
    b = op.apply_adjoint(y)
    Ab = op.apply_adjoint(op.apply(b)) + sp.lam * b
    x1 = (np.vdot(b, b).real / np.vdot(b, Ab).real) * b
    got, it1, _ = O.cg_lmmse(y, op, sp.lam, 1, 0.0)
    assert it1 == 1
    assert np.abs(got - x1).max() <= 1e-14


def test_cg_zero_rhs():
    op = O.TwistedConvChannel(8, 4, [1.0], [1], [1])
    x, it, rel = O.cg_lmmse(np.zeros(32, np.complex64), op, 0.1, 30, 1e-6)
    assert it == 0 and not np.any(x)


@pytest.mark.parametrize("Q", [4, 16, 64, 256])
def test_qam_unit_energy_and_bruteforce_decisions(Q):
    pts = O.qam_points(np.arange(Q), Q)
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) <= 1e-12
    assert np.array_equal(O.qam_decide(pts, Q), np.arange(Q, dtype=np.uint8))
    rng = np.random.default_rng(Q)
    z = pts[rng.integers(0, Q, 4000)] + 0.4 * _rand_c(4000, rng) / math.sqrt(Q)
    z = np.concatenate([z, 3.0 * _rand_c(200, rng)])          # far outside the grid too
    bf = O.qam_decide_bruteforce(z, Q)
    assert np.array_equal(O.qam_decide(z, Q), bf)
    # float32 decisions agree wherever the point is not within rounding of a boundary
    safe = O.decision_margin(z, Q) > 1e-5
    assert np.array_equal(O.qam_decide(z.astype(np.complex64), Q, np.float32)[safe], bf[safe])


def test_qam_ties_go_to_upper_level_and_margin():
    Q, m, s = 16, 4, math.sqrt(10.0)
    # boundary between levels 1 and 2 on both axes sits at 0
    assert O.qam_decide(np.array([0.0 + 0.0j]), Q)[0] == 2 * m + 2
    assert O.qam_decide(np.array([-1e-9 - 1e-9j]), Q)[0] == 1 * m + 1
    assert abs(O.decision_margin(np.array([0.05 + 1j / s]), Q)[0] - 0.05) <= 1e-12


@pytest.mark.parametrize("Q", [4, 16, 64, 256])
def test_gray_bits_neighbours_differ_in_one_bit(Q):
    # the defining property of a Gray map, checked over the whole constellation by brute
    # force: the nearest neighbours of every point (one level apart on one axis) differ in
    # exactly one bit; the map is a bijection onto all bit patterns; and the per-axis code
    # equals the reflected construction G(n) = [0 G(n-1), 1 reverse(G(n-1))]
    m = O.qam_side(Q)
    bits = O.gray_bits(np.arange(Q), Q)
    assert len({tuple(r) for r in bits}) == Q
    pts = O.qam_points(np.arange(Q), Q)
    step = 2.0 / O.qam_scale(Q)
    for a in range(Q):
        for b in range(Q):
            if abs(abs(pts[a] - pts[b]) - step) < 1e-9:
                assert np.count_nonzero(bits[a] != bits[b]) == 1
    codes = [[]]
    for _ in range(int(round(math.log2(m)))):
        codes = [[0] + c for c in codes] + [[1] + c for c in reversed(codes)]
    for i in range(m):
        assert list(O.gray_bits([i * m], Q)[0][:len(codes[0])]) == codes[i]
    assert O.bit_errors([0, 1], [0, 1], Q) == 0


def test_ber_convergence_rule():
    # Eq. ber_convergence on hand-made curves: a negligible fall, a rise, a flat zero curve
    # (zeta guards the division), and a curve that keeps falling fast
    assert O.ber_convergence([0.1, 0.05, 0.0499, 0.04]) == 3
    assert O.ber_convergence([0.1, 0.02, 0.03]) == 3
    assert O.ber_convergence([0.0, 0.0, 0.0]) == 2
    assert O.ber_convergence([0.5, 0.25, 0.125, 0.0625]) == 4
    assert O.ber_convergence([0.2, 0.1999]) == 2


def test_cg_trace_matches_fixed_count_solves():
    # the per-iteration estimates are those of the (pinned) CG stopped after k steps
    rng = np.random.default_rng(77)
    fr = W.small_frame(rng, 16, 8, 3, (0, 4), (-2, 2), qam=16, snr_db=20.0)
    op, _, y = O.received_frame(fr)
    tr = O.cg_lmmse_trace(y, op, fr.spec.lam, 6)
    for k in (1, 2, 6):
        xk, it, _ = O.cg_lmmse(y, op, fr.spec.lam, k, 0.0)
        assert it == k and np.abs(tr[k - 1] - xk).max() <= 1e-12


def test_workload_generator_is_seeded_and_in_range():
    a = W.make_frame_specs("uneven256", nframes=20)
    b = W.make_frame_specs("uneven256", nframes=20)
    for fa, fb in zip(a, b):
        assert (fa.M, fa.N, fa.qam) == (fb.M, fb.N, fb.qam)
        assert np.array_equal(fa.tau, fb.tau) and np.array_equal(fa.h, fb.h)
        assert (fa.M, fa.N) in [(128, 32), (256, 64), (512, 128), (1024, 64)]
        assert 4 <= fa.P <= 16
        assert np.all(fa.tau >= 0) and np.all(fa.tau <= fa.M // 16)
        assert np.all(np.abs(fa.nu) <= fa.N // 8)
        assert len({(int(t), int(v)) for t, v in zip(fa.tau, fa.nu)}) == fa.P
        assert 10.0 <= fa.snr_db <= 30.0 and abs(fa.lam - 10 ** (-fa.snr_db / 10)) < 1e-15
    c2 = W.make_frame_specs("batch64_512x128", nframes=3)
    for sp in c2:
        pw = np.exp(-sp.tau / 8.0)
        assert sp.P == 8 and sp.qam == 16 and np.all(sp.tau <= 32) and np.all(np.abs(sp.nu) <= 8)
        assert pw.shape == (8,)
    fr = W.draw_frame("single_64x16", 0)
    assert fr.sym.shape == (1024,) and fr.noise.shape == (1024,)
    assert abs(np.mean(np.abs(fr.noise) ** 2) / fr.spec.lam - 1.0) < 0.15


# ----------------------------------------------------------------------------------------
# Planted mistakes: a copy of the operator with one plausible error must fail the pins.
# ----------------------------------------------------------------------------------------
def _mutant_dense(M, N, h, tau, nu, mutation):
    E = M * N
    H = np.zeros((E, E), dtype=np.complex128)
    for p in range(len(h)):
        for l in range(N):
            for k in range(M):
                K, L = k - tau[p], l - nu[p]
                n, m = K // M, L // N
                k0, l0 = K - n * M, L - m * N
                qp_l = l if mutation == "row_doppler_in_qp" else l0
                qp = np.exp(2j * np.pi * n * qp_l / N)
                if mutation == "drop_qp":
                    qp = 1.0
                tw_k = k if mutation == "twist_uses_row_delay" else K
                sgn = -1.0 if mutation == "twist_sign" else 1.0
                tw = np.exp(sgn * 2j * np.pi * tw_k * nu[p] / (M * N))
                if mutation == "doppler_sign":
                    l0 = (l + nu[p]) % N
                H[l * M + k, l0 * M + k0] += h[p] * tw * qp
    return H


@pytest.mark.parametrize("mutation", ["none", "row_doppler_in_qp", "drop_qp",
                                      "twist_uses_row_delay", "twist_sign", "doppler_sign"])
def test_pins_catch_planted_mistakes(mutation):
    M, N, tau, nu = 8, 4, [0, 7, -3, 2], [0, 3, -2, -3]
    h = np.array([1.0, 0.5 + 0.5j, -0.3j, 0.7])
    H_eq = O.dense_H_eq_Hdd(M, N, h, tau, nu)
    H_mut = _mutant_dense(M, N, h, tau, nu, mutation)
    err = np.abs(H_mut - H_eq).max()
    if mutation == "none":
        assert err <= 1e-13
    else:
        assert err > 1e-3


def test_fractional_channel_reduces_to_the_operator_and_shifts_exactly():
    # integer delays and Dopplers: the time-domain simulation, taken to the DD domain by the
    # DZT, is the (pinned) DD operator; a fractional delay moves a band-limited tone by the
    # closed-form phase; delays compose and the shift is norm-preserving
    M, N = 8, 4
    rng = np.random.default_rng(91)
    h = _rand_c(3, rng)
    tau, nu = [0, 3, 6], [1, -2, 0]
    x = _rand_c(M * N, rng)
    y_td = O.fractional_td_channel(O.idzt(x, M, N), M, N, h, tau, nu)
    ref = O.TwistedConvChannel(M, N, h, tau, nu).apply(x)
    assert np.abs(O.dzt(y_td, M, N) - ref).max() <= 1e-12
    E = M * N
    i = np.arange(E)
    for f0 in (1, 5, -7):
        tone = np.exp(2j * np.pi * f0 * i / E)
        out = O.fractional_td_channel(tone, M, N, [1.0], [0.37], [0.0])
        assert np.abs(out - tone * np.exp(-2j * np.pi * f0 * 0.37 / E)).max() <= 1e-12
    a = O.fractional_td_channel(O.fractional_td_channel(x, M, N, [1.0], [0.3], [0.0]), M, N,
                                [1.0], [1.45], [0.0])
    b = O.fractional_td_channel(x, M, N, [1.0], [1.75], [0.0])
    assert np.abs(a - b).max() <= 1e-12
    assert abs(np.linalg.norm(b) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)


def test_veh_a_draws_follow_the_profile():
    pk = W.veh_a_packet(np.random.default_rng(5), 128, 32, ndata=2, qam=16, snr_db=20.0)
    # delays of Table vehAProf in samples at B = M * 30 kHz; Dopplers within nu_max / (df / N)
    assert np.allclose(pk.delay_samples, np.array(W.VEH_A_DELAYS_US) * 1e-6 * 128 * 30e3)
    assert np.all(np.abs(pk.doppler_bins) <= 100.0 / (30e3 / 32) + 1e-12)
    assert pk.sym.shape == (2, 128 * 32) and pk.noise.shape == (2, 128 * 32)
    # noise relative to each frame's own mean power: lam per data sample, lam / (MN) for the
    # impulse pilot
    assert abs(np.mean(np.abs(pk.noise) ** 2) / pk.lam - 1.0) < 0.05
    assert abs(np.mean(np.abs(pk.noise_pilot) ** 2) * 128 * 32 / pk.lam - 1.0) < 0.1
