"""Seeded synthetic inputs for LMMSE-CG equalisation of Zak-OTFS frames.

This module draws random numbers only: frame shapes, path tables (integer delay and
Doppler bins, complex gains), QAM symbol indices and white Gaussian noise samples.  It
holds none of the equaliser's arithmetic: it never applies the channel, never maps a
symbol index to a constellation point and never solves anything.  Both the FP64 oracle
and the GPU path consume what it returns and do their own arithmetic on it.

Channel model (paper Sec. III-B, Eq. heff_model): the effective DD channel is a sum of P
Kronecker impulses at integer bins (tau_p, nu_p) with complex gain h_p.  Bins are signed:
tau_p is the delay shift in bins, nu_p the Doppler shift in bins, |tau_p| < M, |nu_p| < N.
Distinct paths occupy distinct (tau, nu) bins (the dominant-path set of Eq. heff_thres is a
set of grid locations), so they are drawn without replacement.

Noise (Sec. V, channel model paragraph): sigma = sqrt(rho_s / gamma) with unit mean
symbol energy and unit mean total path power, so each DD bin gets w ~ CN(0, lam) with
lam = 10^(-SNR_dB/10); the same lam is the scalar noise covariance of Algorithm 1.

Per frame the draws happen in this order from one numpy PCG64 stream: shape, P, paths,
gains, symbol indices, noise.
"""
from __future__ import annotations

import dataclasses
from typing import Iterator, List, Optional

import numpy as np

__all__ = ["FrameSpec", "Frame", "CONFIGS", "make_frame_specs", "draw_frame", "iter_frames",
           "small_frame", "VEH_A_DELAYS_US", "VEH_A_POWERS_DB", "VehAPacket", "veh_a_packet"]


@dataclasses.dataclass
class FrameSpec:
    """Everything about one frame except the bulk symbol and noise draws."""
    M: int
    N: int
    tau: np.ndarray      # int32[P] signed delay bins
    nu: np.ndarray       # int32[P] signed Doppler bins
    h: np.ndarray        # complex128[P] path gains
    qam: int             # constellation size Q (4, 16, 64, 256) or 0 for none
    snr_db: float
    lam: float           # noise variance = scalar LMMSE regulariser
    max_iters: int
    tol: float

    @property
    def P(self) -> int:
        return int(self.tau.shape[0])

    @property
    def E(self) -> int:
        return self.M * self.N


@dataclasses.dataclass
class Frame:
    spec: FrameSpec
    sym: np.ndarray      # int64[E] symbol indices in [0, Q), vector order q = l*M + k
    noise: np.ndarray    # complex128[E] noise samples, vector order q = l*M + k


# ----------------------------------------------------------------------------------------
# Workload presets.  Sizes and distributions follow the five evaluation configurations of
# this implementation; the paper's own experiments use (M, 32) grids with Veh-A fractional
# channels (Sec. V-A), which an integer-bin DD generator stands in for.
# ----------------------------------------------------------------------------------------
CONFIGS = {
    # 1 x (64,16), P=4, delay [0,8], Doppler [-4,4], CN(0,1/P), QPSK, 20 dB, 30 it / 1e-6
    "single_64x16": dict(nframes=1, shapes=[(64, 16)], P=(4, 4), delay=("abs", 8),
                         doppler=("abs", 4), gains="uniform", qam=(4,), snr=(20.0, 20.0),
                         max_iters=30, tol=1e-6, seed=1001),
    # 64 x (512,128), P=8, delay [0,32], Doppler [-8,8], exponential PDP, 16-QAM, 25 dB
    "batch64_512x128": dict(nframes=64, shapes=[(512, 128)], P=(8, 8), delay=("abs", 32),
                            doppler=("abs", 8), gains="exp_pdp", qam=(16,),
                            snr=(25.0, 25.0), max_iters=50, tol=1e-6, seed=1002),
    # 256 frames, (M,N) uniform over four shapes, P in [4,16], delay [0,M/16],
    # Doppler [-N/8,N/8], QPSK / 16-QAM, SNR uniform 10..30 dB
    "uneven256": dict(nframes=256, shapes=[(128, 32), (256, 64), (512, 128), (1024, 64)],
                      P=(4, 16), delay=("frac", 16), doppler=("frac", 8), gains="uniform",
                      qam=(4, 16), snr=(10.0, 30.0), max_iters=50, tol=1e-6, seed=1003),
    # 128 x (1024,256), P=16, delay [0,64], Doppler [-16,16], 64-QAM, 30 dB
    "batch128_1024x256": dict(nframes=128, shapes=[(1024, 256)], P=(16, 16),
                              delay=("abs", 64), doppler=("abs", 16), gains="uniform",
                              qam=(64,), snr=(30.0, 30.0), max_iters=50, tol=1e-6,
                              seed=1005),
}
# Serving stream: frames drawn as in "uneven256"; arrival times are drawn by the server
# benchmark from its own seeded exponential inter-arrival stream (seed 1004 + rate index).
CONFIGS["serving_uneven"] = dict(CONFIGS["uneven256"], seed=1004)

EXP_PDP_DECAY_BINS = 8.0   # tau_s = (max delay) / 4 for the 32-bin delay spread


def _draw_spec(rng: np.random.Generator, cfg: dict) -> FrameSpec:
    shapes = cfg["shapes"]
    M, N = shapes[int(rng.integers(0, len(shapes)))] if len(shapes) > 1 else shapes[0]
    plo, phi = cfg["P"]
    P = int(rng.integers(plo, phi + 1)) if phi > plo else plo
    dkind, dval = cfg["delay"]
    dmax = dval if dkind == "abs" else M // dval
    vkind, vval = cfg["doppler"]
    vmax = vval if vkind == "abs" else N // vval
    n_tau = dmax + 1              # delays 0..dmax
    n_nu = 2 * vmax + 1           # Dopplers -vmax..vmax
    if P > n_tau * n_nu:
        raise ValueError("more paths than distinct bins")
    pick = rng.choice(n_tau * n_nu, size=P, replace=False)
    tau = (pick // n_nu).astype(np.int32)
    nu = (pick % n_nu - vmax).astype(np.int32)
    if cfg["gains"] == "exp_pdp":
        power = np.exp(-tau.astype(np.float64) / EXP_PDP_DECAY_BINS)
        power /= power.sum()
    else:
        power = np.full(P, 1.0 / P)
    g = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    h = np.sqrt(power / 2.0) * g
    qams = cfg["qam"]
    qam = int(qams[int(rng.integers(0, len(qams)))]) if len(qams) > 1 else int(qams[0])
    slo, shi = cfg["snr"]
    snr = float(rng.uniform(slo, shi)) if shi > slo else float(slo)
    lam = 10.0 ** (-snr / 10.0)
    return FrameSpec(M=M, N=N, tau=tau, nu=nu, h=h.astype(np.complex128), qam=qam,
                     snr_db=snr, lam=lam, max_iters=int(cfg["max_iters"]),
                     tol=float(cfg["tol"]))


def _draw_bulk(rng: np.random.Generator, spec: FrameSpec) -> Frame:
    E = spec.E
    sym = rng.integers(0, max(spec.qam, 1), size=E)
    w = rng.standard_normal(E) + 1j * rng.standard_normal(E)
    noise = np.sqrt(spec.lam / 2.0) * w
    return Frame(spec=spec, sym=sym, noise=noise)


def iter_frames(config: str, seed: Optional[int] = None, nframes: Optional[int] = None,
                with_bulk: bool = True) -> Iterator:
    """Yield the frames of a named workload in draw order (Frame, or FrameSpec only)."""
    cfg = CONFIGS[config]
    rng = np.random.default_rng(cfg["seed"] if seed is None else seed)
    n = cfg["nframes"] if nframes is None else nframes
    for _ in range(n):
        spec = _draw_spec(rng, cfg)
        if with_bulk:
            yield _draw_bulk(rng, spec)
        else:
            # keep the stream position identical to the bulk case
            rng.integers(0, max(spec.qam, 1), size=spec.E)
            rng.standard_normal(spec.E)
            rng.standard_normal(spec.E)
            yield spec


def make_frame_specs(config: str, seed: Optional[int] = None,
                     nframes: Optional[int] = None) -> List[FrameSpec]:
    return list(iter_frames(config, seed, nframes, with_bulk=False))


def draw_frame(config: str, index: int, seed: Optional[int] = None) -> Frame:
    """Frame number `index` of a workload (draws and discards the frames before it)."""
    for i, fr in enumerate(iter_frames(config, seed, index + 1)):
        if i == index:
            return fr
    raise IndexError(index)


def small_frame(rng: np.random.Generator, M: int, N: int, P: int, tau_range, nu_range,
                qam: int = 4, snr_db: float = 20.0, max_iters: int = 30,
                tol: float = 1e-6, distinct: bool = True) -> Frame:
    """A frame with explicit shape and inclusive bin ranges, for tests of edge cases.

    tau_range / nu_range are inclusive (lo, hi) intervals of signed bins.
    """
    t_lo, t_hi = tau_range
    v_lo, v_hi = nu_range
    n_tau, n_nu = t_hi - t_lo + 1, v_hi - v_lo + 1
    if distinct:
        pick = rng.choice(n_tau * n_nu, size=P, replace=False)
    else:
        pick = rng.integers(0, n_tau * n_nu, size=P)
    tau = (pick // n_nu + t_lo).astype(np.int32)
    nu = (pick % n_nu + v_lo).astype(np.int32)
    g = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    h = np.sqrt(1.0 / (2.0 * P)) * g
    lam = 10.0 ** (-snr_db / 10.0)
    spec = FrameSpec(M=M, N=N, tau=tau, nu=nu, h=h, qam=qam, snr_db=snr_db, lam=lam,
                     max_iters=max_iters, tol=tol)
    return _draw_bulk(rng, spec)


# ----------------------------------------------------------------------------------------
# Fractional delay-Doppler packets (the paper's channel model, Sec. V, Table vehAProf): the
# ITU Vehicular-A power-delay profile, Doppler nu_p = nu_max cos(2 pi U_p), U_p ~ U(0, 1).
# Delays and Dopplers are fractional on the DD grid.  Only the random draws live here; the
# time-domain channel is applied by the consumer.
# ----------------------------------------------------------------------------------------
VEH_A_DELAYS_US = (0.00, 0.31, 0.71, 1.09, 1.73, 2.51)
VEH_A_POWERS_DB = (0.0, -1.0, -9.0, -10.0, -15.0, -20.0)


@dataclasses.dataclass
class VehAPacket:
    """One packet: a pilot frame and `ndata` data frames through one Veh-A channel.

    delay_samples[p] = tau_p * B with B = M * df (fractional samples); doppler_bins[p] =
    nu_p / (df / N) (fractional Doppler bins); gains h_p ~ CN(0, power_p) with the profile's
    powers normalised to sum 1.  Noise samples are time-domain, with sigma^2 = rho_s / gamma
    taken per frame from that frame's mean signal power rho_s (Sec. V): lam for a data
    frame (unit-energy symbols), lam / (M N) for the pilot frame (one unit impulse)."""
    M: int
    N: int
    df_hz: float
    nu_max_hz: float
    delay_samples: np.ndarray
    doppler_bins: np.ndarray
    h: np.ndarray
    qam: int
    snr_db: float
    lam: float
    sym: np.ndarray          # int64[ndata, M*N] symbol indices, vector order q = l*M + k
    noise_pilot: np.ndarray  # complex128[M*N] time-domain noise of the pilot frame
    noise: np.ndarray        # complex128[ndata, M*N] time-domain noise of the data frames


def veh_a_packet(rng: np.random.Generator, M: int, N: int, ndata: int = 1, df_hz: float = 30e3,
                 nu_max_hz: float = 100.0, qam: int = 4, snr_db: float = 20.0) -> VehAPacket:
    """Draws in this order: path Dopplers U_p, gains, symbols, pilot noise, data noise."""
    B = M * df_hz
    dnu = df_hz / N
    delays = np.asarray(VEH_A_DELAYS_US) * 1e-6 * B
    power = 10.0 ** (np.asarray(VEH_A_POWERS_DB) / 10.0)
    power /= power.sum()
    P = delays.size
    u = rng.uniform(0.0, 1.0, P)
    dopp = nu_max_hz * np.cos(2.0 * np.pi * u) / dnu
    g = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    h = np.sqrt(power / 2.0) * g
    E = M * N
    sym = rng.integers(0, qam, size=(ndata, E))
    lam = 10.0 ** (-snr_db / 10.0)
    wp = np.sqrt(lam / (2.0 * E)) * (rng.standard_normal(E) + 1j * rng.standard_normal(E))
    w = np.sqrt(lam / 2.0) * (rng.standard_normal((ndata, E)) + 1j * rng.standard_normal((ndata, E)))
    return VehAPacket(M=M, N=N, df_hz=df_hz, nu_max_hz=nu_max_hz, delay_samples=delays,
                      doppler_bins=dopp, h=h.astype(np.complex128), qam=qam, snr_db=snr_db,
                      lam=lam, sym=sym, noise_pilot=wp, noise=w)
