"""Scheduling of the continuous-batching server, exercised on the CPU with a
stand-in executor (no GPU): every request is answered exactly once with the rows
of its own flows, in-flight memory never exceeds the budget, cancelled requests
are skipped, and requests are packed several to a micro-batch."""
import threading
import time

import numpy as np
import pytest

from paper_2507_14222_amd import ig
from paper_2507_14222_amd.serve import Server


class FakeExecutor:
    """Scores a flow as (sum of its codes, index of its first max code) after a delay."""

    def __init__(self, cap, d, delay=0.002):
        self.cap, self.d, self.delay = cap, d, delay
        self.launched = []

    def new_slot(self):
        return {"codes": np.zeros((self.cap, self.d), np.uint16), "out": None, "t": 0.0}

    def staging(self, h):
        return h["codes"]

    def launch(self, h, n):
        c = h["codes"][:n].astype(np.int64)
        h["out"] = np.stack([c.sum(axis=1), c.argmax(axis=1)], axis=1)
        h["t"] = time.perf_counter() + self.delay
        self.launched.append(n)

    def ready(self, h):
        return time.perf_counter() >= h["t"]

    def results(self, h, n):
        return h["out"][:n]


def _expected(codes):
    c = codes.astype(np.int64)
    return np.stack([c.sum(axis=1), c.argmax(axis=1)], axis=1)


def test_every_request_gets_its_own_rows():
    d, cap = 5, 300
    exe = FakeExecutor(cap, d)
    rng = np.random.default_rng(0)
    reqs = [rng.integers(0, 9, size=(int(rng.integers(1, 120)), d)).astype(np.uint16) for _ in range(200)]
    with Server(None, n_slots=3, max_batch_flows=cap, d=d, executor=exe) as srv:
        futs = [srv.submit(r) for r in reqs]
        outs = [f.result(timeout=30) for f in futs]
    for r, o in zip(reqs, outs):
        assert np.array_equal(o, _expected(r))
    assert sum(exe.launched) == sum(r.shape[0] for r in reqs)
    assert len(exe.launched) < len(reqs)          # several requests share a micro-batch
    assert max(exe.launched) <= cap


def test_memory_budget_is_respected():
    d, cap = 4, 256
    exe = FakeExecutor(cap, d, delay=0.005)
    budget = 300 * (2 * d + 16)                    # room for 300 flows in flight
    rng = np.random.default_rng(1)
    reqs = [rng.integers(0, 5, size=(int(rng.integers(50, 200)), d)).astype(np.uint16) for _ in range(60)]
    with Server(None, n_slots=4, max_batch_flows=cap, mem_budget_bytes=budget, d=d, executor=exe) as srv:
        futs = [srv.submit(r) for r in reqs]
        for r, f in zip(reqs, futs):
            assert np.array_equal(f.result(timeout=30), _expected(r))
        assert srv.max_in_flight_bytes <= budget


def test_cancelled_request_is_skipped_others_intact():
    d, cap = 3, 64
    exe = FakeExecutor(cap, d, delay=0.02)
    with Server(None, n_slots=1, max_batch_flows=cap, d=d, executor=exe) as srv:
        first = srv.submit(np.ones((64, d), np.uint16))      # occupies the only slot
        f2 = srv.submit(np.full((10, d), 2, np.uint16))
        f3 = srv.submit(np.full((7, d), 3, np.uint16))
        assert f2.cancel()
        assert np.array_equal(first.result(timeout=10), _expected(np.ones((64, d), np.uint16)))
        assert np.array_equal(f3.result(timeout=10), _expected(np.full((7, d), 3, np.uint16)))
    assert f2.cancelled()
    assert sum(exe.launched) == 64 + 7


def test_rejects_bad_requests():
    exe = FakeExecutor(16, 3)
    with Server(None, n_slots=1, max_batch_flows=16, d=3, executor=exe) as srv:
        with pytest.raises(ig.IGError):
            srv.submit(np.zeros((17, 3), np.uint16))
        with pytest.raises(ig.IGError):
            srv.submit(np.zeros((4, 2), np.uint16))
        with pytest.raises(ig.IGError):
            srv.submit(np.zeros((0, 3), np.uint16))


def test_failing_executor_fails_outstanding_requests():
    class Broken(FakeExecutor):
        def launch(self, h, n):
            raise RuntimeError("device lost")

    exe = Broken(8, 2)
    srv = Server(None, n_slots=1, max_batch_flows=8, d=2, executor=exe)
    f = srv.submit(np.zeros((3, 2), np.uint16))
    with pytest.raises(RuntimeError):
        f.result(timeout=10)
    with pytest.raises(RuntimeError):
        srv.close()


def test_concurrent_submitters():
    d, cap = 4, 512
    exe = FakeExecutor(cap, d, delay=0.001)
    rng = np.random.default_rng(2)
    per_thread = [[rng.integers(0, 7, size=(int(rng.integers(1, 300)), d)).astype(np.uint16) for _ in range(40)]
                  for _ in range(4)]
    results = [None] * 4
    with Server(None, n_slots=3, max_batch_flows=cap, d=d, executor=exe) as srv:
        def work(k):
            futs = [srv.submit(r) for r in per_thread[k]]
            results[k] = [f.result(timeout=30) for f in futs]
        ts = [threading.Thread(target=work, args=(k,)) for k in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    for k in range(4):
        for r, o in zip(per_thread[k], results[k]):
            assert np.array_equal(o, _expected(r))


def test_process_settings_are_restored_by_the_last_server():
    """The collector freeze and the switch interval are held while any server runs
    and restored when the last one closes, also when a constructor fails."""
    import gc
    import sys
    if gc.get_freeze_count():
        pytest.skip("objects were frozen before this test")
    switch = sys.getswitchinterval()
    a = Server(None, n_slots=1, max_batch_flows=8, d=2, executor=FakeExecutor(8, 2))
    b = Server(None, n_slots=1, max_batch_flows=8, d=2, executor=FakeExecutor(8, 2), freeze_gc=False)
    c = Server(None, n_slots=1, max_batch_flows=8, d=2, executor=FakeExecutor(8, 2))
    assert gc.get_freeze_count() > 0 and sys.getswitchinterval() <= 0.0005
    with pytest.raises(ValueError):
        Server(None, n_slots=1, max_batch_flows=8, executor=FakeExecutor(8, 2))   # no d
    a.close()
    c.close()
    assert gc.get_freeze_count() == 0          # the last freezing server is gone
    assert sys.getswitchinterval() <= 0.0005   # b still runs
    assert np.array_equal(b.submit(np.ones((2, 2), np.uint16)).result(timeout=10), _expected(np.ones((2, 2))))
    b.close()
    assert sys.getswitchinterval() == switch
