"""FP64 CPU oracle for LMMSE-CG equalisation of Zak-OTFS frames.

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the tests, the smoke check and the
cpu_baseline leg of the benchmark may import or call this module.

Everything here is complex128 / float64 NumPy and follows the paper's definitions
directly, slowly and without fusion:

* the channel operator is the discrete twisted convolution of the effective channel with
  the quasi-periodic extension of the frame (Sec. III-B, Eq. y_channel_DD and its two
  footnotes; the effective channel is the impulse sum of Eq. heff_model);
* three further dense constructions of the same matrix for tiny frames: Eq. Hdd as
  printed, the product form sum_p h_p Pi^tau_p Delta^nu_p of delay and Doppler shift
  operators, and the DZT-conjugated time-domain channel (Eqs. zak, iZak, y_discrete_td);
* the LMMSE solution (Eq. lmmse) by Cholesky on the dense normal equations;
* conjugate gradient (Hestenes-Stiefel) on the normal equations, the iteration of
  Algorithm 1 (Sec. IV-C), with a per-frame relative-residual stop test after the residual
  update;
* hard QAM decisions (Eq. demod), per axis and by brute force, their bits (a Gray map per
  axis) and bit-error counts;
* the BER-driven iteration budget (Eq. ber_convergence) over per-iteration CG estimates;
* the point-pilot channel estimate (Eq. heff) and its Hadamard form (Eq. heff_exp,
  Eq. heff_hadamard), and the dominant-path set by thresholding (Eq. heff_thres).

Conventions (readings of the paper where it leaves a choice open):
* A frame is X[k, l], delay bin k in [0, M), Doppler bin l in [0, N).  The vector form
  is q = l*M + k (Sec. IV-B indexes rows that way); Eq. Hdd's k'N + l' row index is
  re-indexed to it.
* Paths are given by signed bin shifts (tau_p, nu_p) with |tau_p| < M, |nu_p| < N, i.e. the
  pilot reference (K0, L0) is already subtracted.
* The time-domain channel uses the path's Doppler in its phase ramp, exp(j 2 pi nu_p (i -
  tau_p) / (M N)); the printed exponent repeats the delay symbol there.
* Algorithm 1's p^H a_p is real in exact arithmetic; the real part is taken.

Parity pins for every function here live in tests/test_oracle.py; there is no function in
this module whose parity is unpinned.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

__all__ = [
    "vec", "unvec", "TwistedConvChannel", "apply_H", "apply_HH", "dense_from_operator",
    "dense_H_eq_Hdd", "dense_H_shift_ops", "dzt_matrix", "dzt", "idzt", "dense_H_timedomain",
    "cg_lmmse", "lmmse_dense", "qam_side", "qam_scale", "qam_points", "qam_decide",
    "qam_decide_bruteforce", "decision_margin", "pilot_estimate_direct",
    "pilot_estimate_hadamard", "pilot_frame", "threshold_paths", "received_frame", "nmse",
    "gray_bits", "bit_errors", "cg_lmmse_trace", "ber_convergence",
    "fractional_td_channel", "veh_a_received",
]


# ----------------------------------------------------------------------------------------
# vectorisation (Sec. IV-B: row q has delay k_q = <q>_M and Doppler l_q = floor(q / M))
# ----------------------------------------------------------------------------------------
def vec(X: np.ndarray) -> np.ndarray:
    """X[k, l] (shape M x N) -> x[q], q = l*M + k."""
    return np.ascontiguousarray(X.T).reshape(-1)


def unvec(x: np.ndarray, M: int, N: int) -> np.ndarray:
    """x[q] -> X[k, l] with q = l*M + k."""
    return np.asarray(x).reshape(N, M).T


def _check_paths(M, N, h, tau, nu):
    h = np.asarray(h, dtype=np.complex128).reshape(-1)
    tau = np.asarray(tau, dtype=np.int64).reshape(-1)
    nu = np.asarray(nu, dtype=np.int64).reshape(-1)
    if M < 1 or N < 1:
        raise ValueError("M and N must be >= 1")
    if not (h.shape == tau.shape == nu.shape):
        raise ValueError("h, tau, nu must have the same length")
    if np.any(np.abs(tau) >= M) or np.any(np.abs(nu) >= N):
        raise ValueError("need |tau_p| < M and |nu_p| < N")
    return h, tau, nu


# ----------------------------------------------------------------------------------------
# The channel operator by definition: discrete twisted convolution (Eq. y_channel_DD)
# ----------------------------------------------------------------------------------------
class TwistedConvChannel:
    """y = h_eff *_sigma x_qp for an effective channel of P integer-bin impulses.

    Twisted convolution (footnote of Eq. y_channel_DD):
        (a *_sigma b)[k, l] = sum_{k', l'} a[k - k', l - l'] b[k', l'] e^{j 2 pi k' (l - l') / (M N)}.
    With a = h_eff = sum_p h_p delta[k - tau_p] delta[l - nu_p] (Eq. heff_model) the only
    surviving terms are k' = k - tau_p, l' = l - nu_p, so
        y[k, l] = sum_p h_p e^{j 2 pi (k - tau_p) nu_p / (M N)} x_qp[k - tau_p, l - nu_p].
    b is the quasi-periodic extension of the frame (second footnote):
        x_qp[k0 + n M, l0 + m N] = x[k0, l0] e^{j 2 pi n l0 / N}.

    The per-path source indices and unit-modulus factors are tabulated once at
    construction (a cache of the definition, not a rearrangement of it).
    """

    def __init__(self, M: int, N: int, h, tau, nu):
        h, tau, nu = _check_paths(M, N, h, tau, nu)
        self.M, self.N = int(M), int(N)
        self.h, self.tau, self.nu = h, tau, nu
        k = np.arange(M, dtype=np.int64)[:, None]
        l = np.arange(N, dtype=np.int64)[None, :]
        self.terms = []
        for p in range(h.shape[0]):
            K = k - tau[p]                   # raw source delay  k' = k - tau_p   (M, 1)
            L = l - nu[p]                    # raw source Doppler l' = l - nu_p   (1, N)
            n = np.floor_divide(K, M)        # K = k0 + n M
            k0 = K - n * M
            m = np.floor_divide(L, N)        # L = l0 + m N
            l0 = L - m * N
            qp = np.exp(2j * np.pi * (n * l0) / N)                 # quasi-periodic factor
            twist = np.exp(2j * np.pi * (K * nu[p]) / (M * N))     # twisted-conv kernel
            coef = h[p] * twist * qp                                 # (M, N)
            src_k = np.broadcast_to(k0, (M, N))
            src_l = np.broadcast_to(l0, (M, N))
            # source position in vector order (q = l*M + k) for every output position
            src = vec(src_l * M + src_k)
            # each path moves every grid point to exactly one place (a permutation)
            if np.unique(src).size != M * N:
                raise AssertionError("path map is not a permutation")
            self.terms.append((src, vec(coef)))

    @property
    def E(self) -> int:
        return self.M * self.N

    def apply(self, x: np.ndarray) -> np.ndarray:
        """y = H x (x in vector order q = l*M + k)."""
        x = np.asarray(x, dtype=np.complex128).reshape(-1)
        y = np.zeros(self.E, dtype=np.complex128)
        for src, coef in self.terms:
            y += coef * x[src]
        return y

    def apply_adjoint(self, y: np.ndarray) -> np.ndarray:
        """x = H^H y: every term of apply() scattered back with the conjugate factor."""
        y = np.asarray(y, dtype=np.complex128).reshape(-1)
        x = np.zeros(self.E, dtype=np.complex128)
        for src, coef in self.terms:
            # src is a permutation of the grid, so no index repeats within a term
            x[src] += np.conj(coef) * y
        return x


def apply_H(x, M, N, h, tau, nu):
    return TwistedConvChannel(M, N, h, tau, nu).apply(x)


def apply_HH(y, M, N, h, tau, nu):
    return TwistedConvChannel(M, N, h, tau, nu).apply_adjoint(y)


def dense_from_operator(op: TwistedConvChannel) -> np.ndarray:
    """Dense matrix of an operator, column by column (tiny frames only)."""
    E = op.E
    H = np.zeros((E, E), dtype=np.complex128)
    e = np.zeros(E, dtype=np.complex128)
    for j in range(E):
        e[j] = 1.0
        H[:, j] = op.apply(e)
        e[j] = 0.0
    return H


# ----------------------------------------------------------------------------------------
# Eq. Hdd as printed (re-indexed from k'N + l' to q = l*M + k)
# ----------------------------------------------------------------------------------------
def dense_H_eq_Hdd(M, N, h, tau, nu) -> np.ndarray:
    """H[(k', l'), (k, l)] = sum_{n, m} e^{j 2 pi (l' - l - mN)(k + nM) / (MN)}
                                       h_eff[k' - k - nM, l' - l - mN] e^{j 2 pi n l / N}.

    h_eff is the impulse sum of Eq. heff_model, so the (n, m) term is nonzero only when
    k' - k - nM = tau_p and l' - l - mN = nu_p for some path p.
    """
    h, tau, nu = _check_paths(M, N, h, tau, nu)
    kp = np.arange(M)[:, None, None, None]
    lp = np.arange(N)[None, :, None, None]
    k = np.arange(M)[None, None, :, None]
    l = np.arange(N)[None, None, None, :]
    H4 = np.zeros((M, N, M, N), dtype=np.complex128)
    for p in range(h.shape[0]):
        dk = kp - k - tau[p]                       # must equal n M
        dl = lp - l - nu[p]                        # must equal m N
        ok = (np.mod(dk, M) == 0) & (np.mod(dl, N) == 0)
        n = np.floor_divide(dk, M)
        m = np.floor_divide(dl, N)
        phase1 = np.exp(2j * np.pi * ((lp - l - m * N) * (k + n * M)) / (M * N))
        phase2 = np.exp(2j * np.pi * (n * l) / N)
        H4 += np.where(ok, phase1 * h[p] * phase2, 0.0)
    # rows (k', l') -> q' = l' M + k',  cols (k, l) -> q = l M + k
    return H4.transpose(1, 0, 3, 2).reshape(M * N, M * N)


# ----------------------------------------------------------------------------------------
# Product form: H = sum_p h_p Pi^{tau_p} Delta^{nu_p}
# ----------------------------------------------------------------------------------------
def _shift_ops(M, N) -> Tuple[np.ndarray, np.ndarray]:
    """Pi: delay by one bin, (Pi x)[k, l] = x_qp[k - 1, l].
    Delta: Doppler by one bin, (Delta x)[k, l] = e^{j 2 pi k / (M N)} x_qp[k, l - 1]."""
    E = M * N
    Pi = np.zeros((E, E), dtype=np.complex128)
    De = np.zeros((E, E), dtype=np.complex128)
    for l in range(N):
        for k in range(M):
            q = l * M + k
            if k >= 1:
                Pi[q, l * M + (k - 1)] = 1.0
            else:   # x_qp[-1, l] = x[M - 1, l] e^{-j 2 pi l / N}
                Pi[q, l * M + (M - 1)] = np.exp(-2j * np.pi * l / N)
            De[q, ((l - 1) % N) * M + k] = np.exp(2j * np.pi * k / (M * N))
    return Pi, De


def _mpow(A: np.ndarray, e: int) -> np.ndarray:
    if e >= 0:
        return np.linalg.matrix_power(A, e)
    return np.linalg.matrix_power(A.conj().T, -e)     # unitary: A^{-1} = A^H


def dense_H_shift_ops(M, N, h, tau, nu) -> np.ndarray:
    h, tau, nu = _check_paths(M, N, h, tau, nu)
    Pi, De = _shift_ops(M, N)
    H = np.zeros((M * N, M * N), dtype=np.complex128)
    for p in range(h.shape[0]):
        H += h[p] * (_mpow(Pi, int(tau[p])) @ _mpow(De, int(nu[p])))
    return H


# ----------------------------------------------------------------------------------------
# Zak transforms (Eq. zak, Eq. iZak) and the time-domain channel (Eq. y_discrete_td)
# ----------------------------------------------------------------------------------------
def dzt_matrix(M, N) -> np.ndarray:
    """Z[q, i] with Y[k, l] = N^{-1/2} sum_{i'} y[k + i' M] e^{-j 2 pi i' l / N}, q = lM + k."""
    E = M * N
    Z = np.zeros((E, E), dtype=np.complex128)
    for l in range(N):
        for k in range(M):
            for ip in range(N):
                Z[l * M + k, k + ip * M] = np.exp(-2j * np.pi * ip * l / N) / math.sqrt(N)
    return Z


def dzt(y_td: np.ndarray, M, N) -> np.ndarray:
    """Eq. zak, summed directly; returns the DD frame in vector order."""
    y_td = np.asarray(y_td, dtype=np.complex128)
    Y = np.zeros((M, N), dtype=np.complex128)
    for k in range(M):
        for l in range(N):
            s = 0.0j
            for ip in range(N):
                s += y_td[k + ip * M] * np.exp(-2j * np.pi * ip * l / N)
            Y[k, l] = s / math.sqrt(N)
    return vec(Y)


def idzt(x_dd: np.ndarray, M, N) -> np.ndarray:
    """Eq. iZak, summed directly: x[i] = N^{-1/2} sum_l X[<i>_M, l] e^{j 2 pi floor(i/M) l / N}."""
    X = unvec(np.asarray(x_dd, dtype=np.complex128), M, N)
    out = np.zeros(M * N, dtype=np.complex128)
    for i in range(M * N):
        s = 0.0j
        for l in range(N):
            s += X[i % M, l] * np.exp(2j * np.pi * (i // M) * l / N)
        out[i] = s / math.sqrt(N)
    return out


def dense_H_timedomain(M, N, h, tau, nu) -> np.ndarray:
    """Z H_td Z^H with (H_td x)[i] = sum_p h_p e^{j 2 pi nu_p (i - tau_p)/(MN)} x[<i - tau_p>_{MN}]."""
    h, tau, nu = _check_paths(M, N, h, tau, nu)
    E = M * N
    Htd = np.zeros((E, E), dtype=np.complex128)
    for p in range(h.shape[0]):
        for i in range(E):
            Htd[i, (i - tau[p]) % E] += h[p] * np.exp(2j * np.pi * nu[p] * (i - tau[p]) / E)
    Z = dzt_matrix(M, N)
    return Z @ Htd @ Z.conj().T


def fractional_td_channel(x_td, M, N, h, delay_samples, doppler_bins) -> np.ndarray:
    """Time-domain channel with fractional delays and Dopplers (Eq. y_discrete_td without
    its noise term, with the Doppler in the phase ramp as in dense_H_timedomain):
        y[i] = sum_p h_p e^{j 2 pi nu_p (i - tau_p) / (M N)} x(i - tau_p),
    nu_p in Doppler bins and tau_p in samples, both real.  x(t) is the band-limited
    continuation of the frame, periodic over its M N samples (a delay by tau multiplies
    DFT bin f of the frame by e^{-j 2 pi f tau / (M N)}, f taken in the symmetric range
    [-MN/2, MN/2)); for integer tau this is the circular shift of dense_H_timedomain."""
    x = np.asarray(x_td, dtype=np.complex128).reshape(-1)
    E = M * N
    X = np.fft.fft(x)
    f = np.fft.fftfreq(E) * E                  # symmetric bin indices
    i = np.arange(E)
    y = np.zeros(E, dtype=np.complex128)
    for hp, tau, nu in zip(np.asarray(h), np.asarray(delay_samples, dtype=np.float64),
                           np.asarray(doppler_bins, dtype=np.float64)):
        shifted = np.fft.ifft(X * np.exp(-2j * np.pi * f * tau / E))
        y += hp * np.exp(2j * np.pi * nu * (i - tau) / E) * shifted
    return y


def veh_a_received(packet):
    """(received pilot frame, received data frames) in the time domain for a packet of the
    fractional workload: the pilot impulse at (M/2, N/2) and the QAM data frames, each
    taken to the time domain by Eq. iZak, through fractional_td_channel, plus the packet's
    time-domain noise; rounded once to complex64 (what a receiver gets)."""
    M, N = packet.M, packet.N
    chan = lambda xdd: fractional_td_channel(idzt(xdd, M, N), M, N, packet.h,
                                             packet.delay_samples, packet.doppler_bins)
    yp = (chan(pilot_frame(M, N)) + packet.noise_pilot).astype(np.complex64)
    ys = np.stack([(chan(qam_points(packet.sym[d], packet.qam)) + packet.noise[d])
                   for d in range(packet.sym.shape[0])]).astype(np.complex64)
    return yp, ys


# ----------------------------------------------------------------------------------------
# LMMSE by conjugate gradient on the normal equations
# ----------------------------------------------------------------------------------------
def _normal_operator(op: TwistedConvChannel, lam: float):
    """v -> (H^H H + lam I) v, the Hermitian positive definite matrix of Eq. lmmse."""
    return lambda v: op.apply_adjoint(op.apply(v)) + lam * v


def _stop(rho, rho0, k, max_iters, tol):
    """Stop rule: the relative residual sqrt(rho / rho0) has reached tol (when tol > 0), or
    k = max_iters steps were taken.  tol <= 0 is the fixed-count form of Algorithm 1."""
    rel = math.sqrt(rho / rho0)
    return (tol > 0.0 and rel <= tol) or k >= max_iters, rel


def cg_lmmse(y, op: TwistedConvChannel, lam: float, max_iters: int, tol: float):
    """x = (H^H H + lam I)^{-1} H^H y (Eq. lmmse) by the conjugate gradient method of
    Hestenes and Stiefel (1952) for a Hermitian positive definite system A x = b, started
    from x = 0.

    With residual r = b - A x and search direction d, each step minimises the A-norm of the
    error along d: gamma = (r^H r) / (d^H A d), x += gamma d, r -= gamma A d; the next
    direction d = r + ((r^H r)_new / (r^H r)_old) d is A-conjugate to the previous ones.
    d^H A d is real for Hermitian A; its real part is taken.  This is the iteration of
    Algorithm 1 (Sec. IV-C): its c is r, its p is d, its a_p is A d.

    Stop rule (_stop): after the residual update of step k; tol <= 0 runs exactly max_iters
    steps, Algorithm 1's fixed count.  b = H^H y = 0 gives x = 0 after zero steps.

    Returns (x, steps, relative residual sqrt(r^H r / b^H b) at the last step).
    """
    apply_A = _normal_operator(op, lam)
    b = op.apply_adjoint(np.asarray(y, dtype=np.complex128))
    x = np.zeros_like(b)
    r = b.copy()
    rho0 = rho = float(np.vdot(r, r).real)
    if rho0 == 0.0:
        return x, 0, 0.0
    d = r.copy()
    k, rel = 0, 1.0
    while True:
        q = apply_A(d)
        gamma = rho / float(np.vdot(d, q).real)
        x += gamma * d
        r -= gamma * q
        k += 1
        rho_new = float(np.vdot(r, r).real)
        done, rel = _stop(rho_new, rho0, k, max_iters, tol)
        if done:
            return x, k, rel
        d = r + (rho_new / rho) * d
        rho = rho_new


def lmmse_dense(y, H: np.ndarray, lam: float) -> np.ndarray:
    """Eq. lmmse: x = (H^H H + lam I)^{-1} H^H y, via a Cholesky factorisation."""
    A = H.conj().T @ H + lam * np.eye(H.shape[0])
    rhs = H.conj().T @ np.asarray(y, dtype=np.complex128)
    L = np.linalg.cholesky(A)
    z = np.linalg.solve(L, rhs)
    return np.linalg.solve(L.conj().T, z)


# ----------------------------------------------------------------------------------------
# QAM and hard decisions (Eq. demod)
# ----------------------------------------------------------------------------------------
def qam_side(Q: int) -> int:
    m = int(round(math.sqrt(Q)))
    if m * m != Q or m < 2:
        raise ValueError("square QAM only")
    return m


def qam_scale(Q: int) -> float:
    """s such that levels (2i - (m - 1)) / s give unit mean symbol energy."""
    return math.sqrt(2.0 * (Q - 1) / 3.0)


def qam_points(idx, Q: int) -> np.ndarray:
    m = qam_side(Q)
    s = qam_scale(Q)
    idx = np.asarray(idx, dtype=np.int64)
    iI, iQ = idx // m, idx % m
    return ((2 * iI - (m - 1)) + 1j * (2 * iQ - (m - 1))) / s


def qam_decide(x, Q: int, dtype=np.float64) -> np.ndarray:
    """Nearest point per axis: i = clip(floor((v s + m) / 2), 0, m - 1), ties to the upper
    level; index = i_I * m + i_Q.  The arithmetic runs in `dtype` (one rounding per op)."""
    m = qam_side(Q)
    s = dtype(qam_scale(Q))
    x = np.asarray(x)

    def axis(v):
        v = v.astype(dtype)
        t = v * s
        t = t + dtype(m)
        t = t * dtype(0.5)
        i = np.floor(t).astype(np.int64)
        return np.clip(i, 0, m - 1)

    return (axis(x.real) * m + axis(x.imag)).astype(np.uint8)


def qam_decide_bruteforce(x, Q: int) -> np.ndarray:
    """Eq. demod literally: argmin over all constellation points of |x - s|^2."""
    pts = qam_points(np.arange(Q), Q)
    d = np.abs(np.asarray(x, dtype=np.complex128)[:, None] - pts[None, :]) ** 2
    return np.argmin(d, axis=1).astype(np.uint8)


def decision_margin(x, Q: int) -> np.ndarray:
    """Distance (in signal units) from each component to its nearest decision boundary,
    min over the two axes; inf where the component lies beyond the outer levels."""
    m = qam_side(Q)
    s = qam_scale(Q)
    x = np.asarray(x, dtype=np.complex128)

    def axis(v):
        u = v * s + m                     # boundaries at even integers 2..2(m-1)
        nearest = np.clip(2.0 * np.round(u / 2.0), 2.0, 2.0 * (m - 1))
        return np.abs(u - nearest) / s

    return np.minimum(axis(x.real), axis(x.imag))


def gray_bits(idx, Q: int) -> np.ndarray:
    """Bits of square-QAM symbol indices i_I * m + i_Q (Eq. demod's demapping to bits, which
    the paper leaves unspecified; reading: a reflected Gray code per axis).  Each axis
    index i becomes g = i XOR (i >> 1) on log2(m) bits, most significant first; a symbol's
    bits are the in-phase axis's followed by the quadrature axis's.  Returns uint8 of shape
    (len(idx), 2 log2(m))."""
    m = qam_side(Q)
    b = int(round(math.log2(m)))
    idx = np.asarray(idx, dtype=np.int64).reshape(-1)
    out = np.zeros((idx.size, 2 * b), dtype=np.uint8)
    for axis, val in enumerate((idx // m, idx % m)):
        g = val ^ (val >> 1)
        for j in range(b):
            out[:, axis * b + j] = (g >> (b - 1 - j)) & 1
    return out


def bit_errors(sym_hat, sym_tx, Q: int) -> int:
    """Number of differing bits between decided and transmitted symbols (gray_bits)."""
    return int(np.count_nonzero(gray_bits(sym_hat, Q) != gray_bits(sym_tx, Q)))


def cg_lmmse_trace(y, op: TwistedConvChannel, lam: float, iters: int):
    """The estimates after each of `iters` conjugate-gradient steps (the method of cg_lmmse
    with a fixed count, Algorithm 1's form): a list whose entry k-1 is x after step k."""
    apply_A = _normal_operator(op, lam)
    b = op.apply_adjoint(np.asarray(y, dtype=np.complex128))
    x = np.zeros_like(b)
    r = b.copy()
    rho = float(np.vdot(r, r).real)
    out = []
    if rho == 0.0:
        return [x.copy() for _ in range(iters)]
    d = r.copy()
    for _ in range(iters):
        q = apply_A(d)
        gamma = rho / float(np.vdot(d, q).real)
        x = x + gamma * d
        r = r - gamma * q
        out.append(x.copy())
        rho_new = float(np.vdot(r, r).real)
        d = r + (rho_new / rho) * d
        rho = rho_new
    return out


def ber_convergence(ber, eta: float = 1e-2, zeta: float = 1e-12) -> int:
    """Convergence iteration of a BER curve (Eq. ber_convergence): with ber[k-1] the BER
    after k iterations, the signed relative change r_k = (BER_{k-1} - BER_k) /
    max(BER_{k-1}, zeta); the BER has converged at the first k >= 2 with r_k < eta (a rise
    or a negligible fall).  Returns that k, or len(ber) when no k qualifies."""
    ber = [float(v) for v in ber]
    for k in range(2, len(ber) + 1):
        prev, cur = ber[k - 2], ber[k - 1]
        if (prev - cur) / max(prev, zeta) < eta:
            return k
    return len(ber)


# ----------------------------------------------------------------------------------------
# Point-pilot channel estimate (Eq. heff; Eq. heff_exp with Eq. heff_hadamard)
# ----------------------------------------------------------------------------------------
def pilot_estimate_direct(y_pilot, M, N) -> dict:
    """h_hat[k, l] = Y[k + M/2, l + N/2] e^{-j pi l / N}, -M/2 <= k < M/2, -N/2 <= l < N/2.
    Returned as {(k, l): value}."""
    Y = unvec(np.asarray(y_pilot, dtype=np.complex128), M, N)
    out = {}
    for k in range(-(M // 2), M - M // 2):
        for l in range(-(N // 2), N - N // 2):
            out[(k, l)] = Y[k + M // 2, l + N // 2] * np.exp(-1j * np.pi * l / N)
    return out


def pilot_estimate_hadamard(y_pilot, M, N) -> np.ndarray:
    """h_hat = Y (Hadamard) E_twist, E_twist[k, l] = e^{-j 2 pi K0 (l - L0) / (M N)}, on the
    received grid: entry (k, l) estimates the path at bin (k - K0, l - L0)."""
    K0, L0 = M // 2, N // 2
    Y = unvec(np.asarray(y_pilot, dtype=np.complex128), M, N)
    l = np.arange(N)[None, :]
    Et = np.exp(-2j * np.pi * K0 * (l - L0) / (M * N))
    return Y * Et


def pilot_frame(M, N) -> np.ndarray:
    """The pilot frame: one unit impulse at (K0, L0) = (M/2, N/2) in the DD grid (Sec. III,
    channel estimation), in vector order."""
    d = np.zeros((M, N), dtype=np.complex128)
    d[M // 2, N // 2] = 1.0
    return vec(d)


def threshold_paths(h_grid, theta: float, dtype=np.float64):
    """Dominant paths of an estimated effective channel (Eq. heff_thres): the bins whose
    magnitude exceeds theta, with gain h_p = h_hat[k_p, l_p].

    h_grid: the Hadamard-form estimate on the received grid (pilot_estimate_hadamard),
    entry (k, l) standing for the path at shifts (tau, nu) = (k - K0, l - L0).  The test
    |h| > theta is taken as |h|^2 > theta^2 in `dtype` on the estimate rounded to that
    precision (a float decision has to be taken in one precision to compare two
    implementations).  Returns (tau, nu, h) in vector order q = l*M + k."""
    H = np.asarray(h_grid)
    M, N = H.shape
    K0, L0 = M // 2, N // 2
    tau, nu, gain = [], [], []
    for l in range(N):
        for k in range(M):
            v = H[k, l]
            re, im = dtype(np.real(v)), dtype(np.imag(v))
            if re * re + im * im > dtype(theta) * dtype(theta):
                tau.append(k - K0)
                nu.append(l - L0)
                gain.append(v)
    return (np.array(tau, dtype=np.int64), np.array(nu, dtype=np.int64),
            np.array(gain, dtype=np.complex128))


# ----------------------------------------------------------------------------------------
# helpers for tests and the benchmark's CPU leg
# ----------------------------------------------------------------------------------------
def received_frame(frame) -> Tuple[TwistedConvChannel, np.ndarray, np.ndarray]:
    """(operator, transmitted x, received y rounded once to complex64) for a workload frame
    (Eq. eq_lin_sys: y = H x + w)."""
    sp = frame.spec
    op = TwistedConvChannel(sp.M, sp.N, sp.h, sp.tau, sp.nu)
    x = qam_points(frame.sym, sp.qam)
    y = op.apply(x) + frame.noise
    return op, x, y.astype(np.complex64)


def nmse(est, ref) -> float:
    ref = np.asarray(ref, dtype=np.complex128)
    est = np.asarray(est, dtype=np.complex128)
    den = float(np.vdot(ref, ref).real)
    num = float(np.vdot(est - ref, est - ref).real)
    return num / den if den > 0 else num
