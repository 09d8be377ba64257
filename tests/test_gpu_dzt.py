"""GPU parity of the discrete Zak transform on the matrix cores (otfs_dzt, Eq. zak as the
batched GEMM of Eq. zak_gemm) and of its inverse (Eq. iZak) against the oracle's direct
sums: every output of small frames, a sample of outputs of large ones, and the round trip."""
import math

import numpy as np
import pytest

import oracle as O
from helpers import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def otfs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02266_amd as m
    m.lib()
    return m


def _rand(rng, n):
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)).astype(np.complex64)


def _tol(N, x):
    # FP32 products and sums of N terms of size <= max|x| / sqrt(N)
    return 4e-7 * math.sqrt(N) * np.abs(x).max() * 4


@pytest.mark.parametrize("M,N,nf", [(64, 16, 3), (128, 32, 2), (37, 11, 2), (8, 4, 1), (1, 5, 2),
                                    (300, 12, 1)])
def test_dzt_matches_direct_sums(otfs, M, N, nf):
    rng = np.random.default_rng(M * 1000 + N)
    x = _rand(rng, nf * M * N)
    say("dzt", M, N, nf)
    y = otfs.dzt(to_dev(x), M, N).cpu().numpy()
    xb = otfs.dzt(to_dev(x), M, N, inverse=True).cpu().numpy()
    for f in range(nf):
        sl = slice(f * M * N, (f + 1) * M * N)
        ref = O.dzt(x[sl].astype(np.complex128), M, N)
        assert np.abs(y[sl] - ref).max() <= _tol(N, x[sl]), f
        refi = O.idzt(x[sl].astype(np.complex128), M, N)
        assert np.abs(xb[sl] - refi).max() <= _tol(N, x[sl]), f


def test_dzt_large_frames_sampled_and_round_trip(otfs):
    M, N, nf = 1024, 256, 4
    rng = np.random.default_rng(5)
    x = _rand(rng, nf * M * N)
    say("dzt", M, N, nf)
    xd = to_dev(x)
    y = otfs.dzt(xd, M, N)
    back = otfs.dzt(y, M, N, inverse=True).cpu().numpy()
    y = y.cpu().numpy()
    assert np.abs(back - x).max() <= 4 * _tol(N, x)           # unitary: IDZT(DZT(x)) = x
    picks = rng.integers(0, nf * M * N, 2000)
    i = np.arange(N)
    for q in picks:
        f, r = divmod(int(q), M * N)
        l, k = divmod(r, M)
        xs = x[f * M * N:(f + 1) * M * N].astype(np.complex128)
        ref = np.sum(xs[k + i * M] * np.exp(-2j * np.pi * i * l / N)) / math.sqrt(N)   # Eq. zak
        assert abs(y[q] - ref) <= _tol(N, xs), (f, k, l)


def test_dzt_rejects_bad_arguments(otfs):
    import torch
    x = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(otfs.OtfsError):
        otfs.dzt(x, 8, 8, out=x)
    with pytest.raises(otfs.OtfsError):
        otfs.dzt(torch.zeros(16384 * 2, dtype=torch.complex64, device="cuda"), 2, 16384)
