"""Host-side checks of libotfs that need no GPU: it loads, exports every function the
C header declares, and validates plans on the host before any device work."""
import ctypes

import numpy as np
import pytest

import paper_2604_02266_amd as otfs


@pytest.fixture(scope="module")
def L():
    return otfs.lib()


def test_exports_every_declared_symbol(L):
    names = otfs.header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), f"libotfs.so does not export {n}"


class _F:
    def __init__(self, M, N, tau, nu, h, lam=0.01, qam=4):
        self.M, self.N, self.tau, self.nu, self.h, self.lam, self.qam = M, N, tau, nu, h, lam, qam


def _plan(frames, **kw):
    return otfs.Plan(frames, bind=False, **kw)


def test_plan_is_host_only_and_sizes_workspace():
    fr = [_F(64, 16, [0, 3], [1, -2], np.array([1 + 0j, 0.5j])),
          _F(8, 4, [7, -7], [3, -3], np.array([0.3, -0.2]))]
    p = _plan(fr)
    nbytes, ne = p.workspace_bytes()
    assert ne == 64 * 16 + 8 * 4
    assert nbytes >= 5 * 8 * ne        # c, p0, p1, t, a
    info = p.info()
    assert info.nframes == 2 and info.total_elems == ne and info.max_paths == 2
    p.close()


@pytest.mark.parametrize("bad,msg", [
    (_F(0, 4, [0], [0], np.array([1.0])), "M and N"),
    (_F(8, 4, [8], [0], np.array([1.0])), "|delay| < M"),
    (_F(8, 4, [-8], [0], np.array([1.0])), "|delay| < M"),
    (_F(8, 4, [0], [4], np.array([1.0])), "|doppler| < N"),
    (_F(8, 4, [0], [0], np.array([np.nan])), "not finite"),
    (_F(8, 4, [0], [0], np.array([1.0]), lam=-1.0), "noise_var"),
    (_F(8, 4, [0], [0], np.array([1.0]), qam=8), "qam"),
    (_F(8, 4, [0] * 65, [0] * 65, np.ones(65)), "P must be"),
])
def test_invalid_frames_are_rejected_on_host(bad, msg):
    with pytest.raises(otfs.OtfsError) as ei:
        _plan([bad])
    assert ei.value.status == otfs.E_INVAL
    assert msg in str(ei.value)


def test_invalid_options_are_rejected():
    fr = [_F(8, 4, [1], [1], np.array([1.0]))]
    for kw, msg in [(dict(max_iters=0), "max_iters"), (dict(rel_tol=-1.0), "rel_tol"),
                    (dict(refresh_every=-2), "refresh_every"), (dict(flags=1 << 20), "flag")]:
        with pytest.raises(otfs.OtfsError) as ei:
            _plan(fr, **kw)
        assert ei.value.status == otfs.E_INVAL and msg in str(ei.value)
    # every documented flag is accepted
    for f in (otfs.NO_LDS_RESIDENT, otfs.SPLIT_DIRECTION, otfs.AGENT_BARRIER,
              otfs.TIME_KERNEL, otfs.D_STORED_C64, otfs.D_STORED_BF16, otfs.LDS_GATHER):
        _plan(fr, flags=f)
    with pytest.raises(otfs.OtfsError):
        _plan(fr, flags=1 << 9)
    # the two stored tables exclude each other
    with pytest.raises(otfs.OtfsError) as ei:
        _plan(fr, flags=otfs.D_STORED_C64 | otfs.D_STORED_BF16)
    assert ei.value.status == otfs.E_INVAL and "exclude" in str(ei.value)


def test_stored_tables_size_the_workspace():
    # P x E entries of 4 (bf16 pair) or 8 (complex64) bytes on top of the on-the-fly plan
    fr = [_F(64, 16, [1, 2, 3], [0, 1, -1], np.array([1.0, 0.5, 0.25]))]
    base = _plan(fr).workspace_bytes()[0]
    bf = _plan(fr, flags=otfs.D_STORED_BF16).workspace_bytes()[0]
    c64 = _plan(fr, flags=otfs.D_STORED_C64).workspace_bytes()[0]
    assert bf - base >= 3 * 1024 * 4 and bf - base < 3 * 1024 * 4 + 512
    assert c64 - base >= 3 * 1024 * 8 and c64 - base < 3 * 1024 * 8 + 512


def test_empty_batch_and_unbound_use(L):
    p = _plan([])
    assert p.workspace_bytes()[1] == 0
    # an unbound plan refuses to run (host check, nothing enqueued)
    fr = [_F(8, 4, [1], [1], np.array([1.0]))]
    q = _plan(fr)
    st = L.otfs_lmmse_cg(q._h, ctypes.c_void_p(1), ctypes.c_void_p(2), None, None, None)
    assert st == otfs.E_STATE and "not bound" in otfs.last_error()


def test_tiling_changes_workspace():
    fr = [_F(512, 128, [0, 3], [1, -2], np.array([1 + 0j, 0.5j]))]
    p = _plan(fr)
    p.set_tiling(4096, 0, rebind=False)
    assert p.info().tile_elems == 4096
    p.set_tiling(65536, 0, rebind=False)
    assert p.info().tile_elems == 65536
    with pytest.raises(otfs.OtfsError):
        p.set_tiling(-1, 0, rebind=False)


def test_ber_profile_rule_matches_the_oracle():
    # the profiler's convergence rule (product code) against the oracle's statement of
    # Eq. ber_convergence, on random and hand-made BER curves
    import oracle as O
    from paper_2604_02266_amd import ber_profile
    rng = np.random.default_rng(3)
    curves = [[0.1, 0.05, 0.0499, 0.04], [0.1, 0.02, 0.03], [0.0, 0.0, 0.0], [0.5, 0.25, 0.125]]
    curves += [list(np.sort(rng.uniform(0, 0.2, 12))[::-1] * rng.uniform(0.9, 1.1, 12))
               for _ in range(50)]
    for c in curves:
        assert ber_profile.convergence_iteration(c) == O.ber_convergence(c)


def test_build_stamp_matches_the_sources():
    # the library carries the hash of the sources it was compiled from; the loader compares
    # it with this tree, so a stale build cannot pass for the current code
    info = otfs.build_info()
    assert len(info["source_sha"]) == 16 and info["arch"].startswith("gfx")
    assert info["current"] is True, info
