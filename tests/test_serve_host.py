"""Host-side logic of the serving engine (admission, traces, summaries); no GPU."""
import collections
import time

import numpy as np
import pytest

from paper_2208_04726_amd import serve


def _req(rid, N, M, E, arrival=0.0):
    z = lambda *s: np.zeros(s)
    return serve.Request(rid=rid, stream=0, arrival=arrival, n_fixed=2, intrinsics=z(4),
                         poses=z(N, 7), patches=z(M, 3), anchor=np.zeros(M, np.int32),
                         kk=np.zeros(E, np.int32), jj=np.zeros(E, np.int32),
                         targets=z(E, 2).astype(np.float32), weights=z(E, 2).astype(np.float32))


def test_admit_takes_fifo_prefix_that_fits():
    cap = serve.Capacity(windows=8, frames=40, patches=1000, edges=10_000)
    q = collections.deque([_req(0, 10, 200, 3000), _req(1, 20, 300, 3000), _req(2, 15, 100, 1000),
                           _req(3, 5, 10, 10)])
    b = serve.admit(q, cap)
    # request 2 would exceed 40 frames; admission stops there (no overtaking)
    assert [r.rid for r in b] == [0, 1]
    assert [r.rid for r in q] == [2, 3]
    b = serve.admit(q, cap)
    assert [r.rid for r in b] == [2, 3] and not q


@pytest.mark.parametrize("limit", ["windows", "patches", "edges"])
def test_admit_respects_every_capacity(limit):
    kw = dict(windows=100, frames=10_000, patches=10_000, edges=100_000)
    kw[limit] = {"windows": 3, "patches": 250, "edges": 2500}[limit]
    cap = serve.Capacity(**kw)
    q = collections.deque(_req(i, 8, 100, 1000) for i in range(10))
    b = serve.admit(q, cap)
    assert len(b) == {"windows": 3, "patches": 2, "edges": 2}[limit]
    F = sum(r.shape[0] for r in b)
    P = sum(r.shape[1] for r in b)
    E = sum(r.shape[2] for r in b)
    assert len(b) <= cap.windows and F <= cap.frames and P <= cap.patches and E <= cap.edges


def test_admit_empty_and_fits():
    cap = serve.Capacity(windows=2, frames=30, patches=100, edges=100, frames_per_window=22)
    assert serve.admit(collections.deque(), cap) == []
    assert cap.fits(_req(0, 22, 100, 100))
    assert not cap.fits(_req(0, 23, 10, 10))
    assert not cap.fits(_req(0, 10, 101, 10))
    # a request that cannot fit is never admitted (and blocks the queue, so the
    # server rejects such requests before queueing them)
    q = collections.deque([_req(0, 10, 101, 10)])
    assert serve.admit(q, cap) == [] and len(q) == 1


def test_poisson_trace_is_seeded_and_has_the_rate():
    pool = [_req(i, 8, 10, 10) for i in range(5)]
    a = serve.poisson_trace(pool, 4000, rate=2000.0, seed=3)
    b = serve.poisson_trace(pool, 4000, rate=2000.0, seed=3)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) >= 0)
    assert abs(len(t) / t[-1] - 2000.0) < 100.0       # ~1/sqrt(4000) relative spread
    assert [r.rid for r in a] == list(range(4000))
    sid = np.array([r.stream for r in a])
    assert sid.min() >= 0 and sid.max() < 64
    closed = serve.poisson_trace(pool, 10, rate=float("inf"))
    assert all(r.arrival == 0.0 for r in closed)


def test_latency_summary():
    res = {i: serve.Result(i, None, None, 0, latency=(i + 1) * 1e-3) for i in range(100)}
    s = serve.latency_summary(res, skip=0)
    assert s["n"] == 100 and abs(s["p50_ms"] - 50.5) < 1e-9 and abs(s["mean_ms"] - 50.5) < 1e-9
    s = serve.latency_summary(res, skip=90)
    assert s["n"] == 10 and s["p99_ms"] <= 100.0


class _FakeSlotless(serve.BatchedServer):
    """BatchedServer without slots (no GPU): every fitting request stays
    pending, so only the rejection path answers."""

    def __init__(self, cap):
        self.cap = cap
        self.slots = []
        self.batches = 0
        self.batch_sizes = []


def test_oversize_request_is_rejected_alone():
    from paper_2208_04726_amd import native
    cap = serve.Capacity(windows=4, frames=44, patches=200, edges=2000, frames_per_window=22)
    big = _req(7, 23, 10, 10)          # more frames than a window may hold
    wide = _req(8, 10, 500, 10)        # more patches than a slot holds
    srv = _FakeSlotless(cap)
    res = srv._run([big, wide], clock=iter(np.arange(0.0, 100.0, 0.01)).__next__)
    assert set(res) == {7, 8}
    for r in res.values():
        assert r.status == native.BA_E_CAPACITY
    assert res[7].poses.shape == (23, 7) and res[8].depth.shape == (500,)


class _FakeDriver:
    """Records the frame ids of every step (no GPU)."""

    def __init__(self, S, step_time=0.0):
        self.S, self.calls, self.step_time = S, [], step_time

    def step(self, fid):
        self.calls.append(np.array(fid).copy())
        if self.step_time:
            time.sleep(self.step_time)


def test_stream_server_steps_each_stream_in_order_and_batches():
    from paper_2208_04726_amd.serve import StreamServer, frame_trace
    reqs = frame_trace(5, 7, fps=4000.0, seed=1)
    drv = _FakeDriver(5, step_time=1e-3)
    res = StreamServer(drv).run(reqs)
    assert sorted(res) == list(range(len(reqs)))
    per = {s: [] for s in range(5)}
    step_of = {}
    for k, fid in enumerate(drv.calls):
        for s in range(5):
            if fid[s] >= 0:
                per[s].append(int(fid[s]))
                step_of[(s, int(fid[s]))] = k
    assert all(per[s] == list(range(7)) for s in range(5))           # in order, once each
    assert max(r.batch for r in res.values()) > 1                     # frames were stepped together
    assert len(drv.calls) < len(reqs)
    for r in res.values():
        assert r.latency >= 0
        assert r.batch == int((drv.calls[step_of[(r.stream, r.frame)]] >= 0).sum())


def test_plain_stream_server_is_one_frame_per_step_in_arrival_order():
    from paper_2208_04726_amd.serve import PlainStreamServer, frame_trace
    reqs = frame_trace(3, 4, fps=5000.0, seed=2)
    drivers = [_FakeDriver(1) for _ in range(3)]
    res = PlainStreamServer(drivers).run(reqs)
    assert sorted(res) == list(range(len(reqs)))
    for s in range(3):
        assert [int(c[0]) for c in drivers[s].calls] == list(range(4))
    assert all(r.batch == 1 for r in res.values())
