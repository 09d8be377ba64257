"""Serving-loop host logic on a dry-run server (device -1): admission in arrival order under
the pool budget, tickets, statistics and argument checks.  No GPU work is done."""
import time

import numpy as np
import pytest

import paper_2604_02266_amd as otfs

from helpers import SpecLike


def _frame(M=64, N=16, qam=4):
    return SpecLike(M, N, [0, 3], [1, -2], [1.0, 0.4j], lam=0.05, qam=qam)


def _y(fr):
    return np.zeros(fr.E, dtype=np.complex64)


def _dry(pool_bytes=64 << 20, **kw):
    return otfs.Server(pool_bytes, device=-1, **kw)


def test_dry_run_completes_frames():
    with _dry(max_iters=25, step_iters=10) as s:
        frames = [_frame(), _frame(32, 8, qam=16), _frame(128, 4, qam=0)]
        tickets = [s.submit(f, _y(f)) for f in frames]
        assert tickets == sorted(tickets) and len(set(tickets)) == 3
        for t, f in zip(tickets, frames):
            x, sym, st, lat = s.wait(t, f)
            assert st.status == otfs.FRAME_DRYRUN
            assert st.iters == 25
            assert np.all(x == 0)
            assert (sym is None) == (f.qam == 0)
            assert lat >= 0.0
        ss = s.stats()
        assert ss.submitted == 3 and ss.completed == 3
        assert ss.queued == 0 and ss.active == 0 and ss.pool_bytes_in_use == 0
        # three steps (10 + 10 + 5 iterations) when all three are admitted together
        assert ss.steps >= 3


def test_ticket_is_forgotten_after_poll():
    with _dry() as s:
        f = _frame()
        t = s.submit(f, _y(f))
        s.wait(t, f)
        with pytest.raises(otfs.OtfsError) as ei:
            s.poll(t, f)
        assert ei.value.status == otfs.E_NOTFOUND
        with pytest.raises(otfs.OtfsError) as ei:
            s.poll(12345, f)
        assert ei.value.status == otfs.E_NOTFOUND


def test_pool_budget_serialises_admission_in_arrival_order():
    f = _frame()
    with _dry(max_iters=40, step_iters=1) as probe:
        fb, cb = probe.frame_bytes(f)
    assert fb >= 7 * 8 * f.E and cb > 0
    # room for exactly two frames at once
    # (long dry-run frames, so that all six are queued before the first two finish)
    with _dry(pool_bytes=cb + 2 * fb + 100, max_iters=20000, step_iters=1) as s:
        tickets = [s.submit(f, _y(f)) for _ in range(6)]
        lat = []
        for t in tickets:
            lat.append(s.wait(t, f)[3])
        ss = s.stats()
        assert ss.completed == 6
        assert ss.pool_bytes_peak <= 2 * fb
        assert ss.pool_bytes_peak > fb
        # admitted two at a time, one iteration per step: at least three rounds of steps
        assert ss.steps >= 3 * 20000
    # arrival order is kept: later tickets never finish before earlier ones (all were
    # submitted at about the same time, so latency grows with the ticket)
    assert all(b >= a * 0.5 for a, b in zip(lat, lat[1:]))


def test_frame_larger_than_pool_is_rejected():
    f = _frame()
    with _dry() as probe:
        fb, cb = probe.frame_bytes(f)
    with _dry(pool_bytes=cb + fb - 1) as s:
        with pytest.raises(otfs.OtfsError) as ei:
            s.submit(f, _y(f))
        assert ei.value.status == otfs.E_BUDGET
        small = _frame(8, 4)
        t = s.submit(small, _y(small))
        assert s.wait(t, small)[2].status == otfs.FRAME_DRYRUN


def test_create_argument_checks():
    with pytest.raises(otfs.OtfsError) as ei:
        _dry(step_iters=0)
    assert ei.value.status == otfs.E_INVAL
    with pytest.raises(otfs.OtfsError) as ei:
        _dry(flags=otfs.Y_BF16)
    assert ei.value.status == otfs.E_UNSUPPORTED
    with pytest.raises(otfs.OtfsError) as ei:
        _dry(pool_bytes=1024)
    assert ei.value.status == otfs.E_BUDGET
    with pytest.raises(otfs.OtfsError) as ei:
        otfs.Server(64 << 20, device=-2)
    assert ei.value.status == otfs.E_INVAL


def test_submit_validates_frames():
    with _dry() as s:
        bad = SpecLike(8, 4, [8], [0], [1.0])
        with pytest.raises(otfs.OtfsError) as ei:
            s.submit(bad, np.zeros(32, np.complex64))
        assert ei.value.status == otfs.E_INVAL
        with pytest.raises(ValueError):
            s.submit(_frame(), np.zeros(3, np.complex64))


def test_many_frames_mixed_shapes():
    rng = np.random.default_rng(7)
    with _dry(max_iters=12, step_iters=5) as s:
        frames, tickets = [], []
        for i in range(200):
            M = int(rng.choice([8, 16, 64, 128]))
            N = int(rng.choice([4, 8, 16]))
            fr = SpecLike(M, N, [0, 1], [0, 1], [1.0, 0.3], qam=4)
            frames.append(fr)
            tickets.append(s.submit(fr, _y(fr)))
        for t, fr in zip(tickets, frames):
            assert s.wait(t, fr)[2].iters == 12
        assert s.stats().completed == 200


def test_free_with_frames_in_flight():
    s = _dry(max_iters=10 ** 6, step_iters=1)
    f = _frame()
    for _ in range(5):
        s.submit(f, _y(f))
    time.sleep(0.01)
    s.close()          # drops queued and running frames, joins the scheduler


def test_submit_many_and_poll_many():
    with _dry(max_iters=12, step_iters=4) as s:
        frames = [_frame(), _frame(32, 8, qam=16), _frame(128, 4, qam=0)] * 3
        prep = [s.prepare(f) for f in frames]
        tickets = s.submit_many(prep, [_y(f) for f in frames])
        assert tickets == sorted(tickets) and len(set(tickets)) == len(frames)
        outs = [(np.full(f.E, 1 + 1j, dtype=np.complex64), np.full(f.E, 7, dtype=np.uint8))
                for f in frames]
        left = list(range(len(frames)))
        t_end = time.monotonic() + 30.0
        while left:
            res = s.poll_many([tickets[i] for i in left], [outs[i] for i in left])
            nxt = []
            for i, r in zip(left, res):
                if r is None:
                    nxt.append(i)
                    continue
                st, lat = r
                assert st.status == otfs.FRAME_DRYRUN and st.iters == 12 and lat >= 0.0
                assert np.all(outs[i][0] == 0)
                # a frame without a constellation leaves the decision buffer alone
                assert np.all(outs[i][1] == (7 if frames[i].qam == 0 else 0))
            left = nxt
            assert time.monotonic() < t_end
            time.sleep(1e-3)
        ss = s.stats()
        assert ss.submitted == len(frames) and ss.completed == len(frames)
        # every ticket was forgotten by the batched poll
        with pytest.raises(otfs.OtfsError) as ei:
            s.poll_many([tickets[0]], [outs[0]])
        assert ei.value.status == otfs.E_NOTFOUND


def test_submit_many_rejects_the_whole_batch():
    with _dry() as s:
        good = _frame()
        bad = SpecLike(64, 16, [0, 3], [1, -2], [1.0, 0.5], lam=0.05, qam=5)   # no such QAM
        with pytest.raises(otfs.OtfsError):
            s.submit_many([good, bad], [_y(good), _y(bad)])
        assert s.stats().submitted == 0
        with pytest.raises(ValueError):
            s.submit_many([good], [np.zeros(good.E - 1, dtype=np.complex64)])
