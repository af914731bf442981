"""Host logic of the serving loop (admission by budget, continuous batching,
retirement) against a fake backend whose batches take a fixed wall time."""
import time

import numpy as np
import pytest

from paper_1611_04474_amd.serving import Item, run_policy


class FakeBackend:
    def __init__(self, batch_s=0.002):
        self.batch_s = batch_s
        self.events = []          # (kind, time, payload)
        self.resident = 0
        self.max_resident = 0
        self.inflight = 0
        self.max_inflight = 0

    def admit(self, it):
        self.resident += it.bytes
        self.max_resident = max(self.max_resident, self.resident)
        self.events.append(("admit", time.perf_counter(), it.rid))
        return {"item": it}

    def launch(self, handles):
        t = time.perf_counter()
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        rids = [h["item"].rid for h in handles]
        self.events.append(("launch", t, rids))
        # batches on one stream run one after another
        prev_end = max([b["end"] for b in getattr(self, "_batches", [])] + [t])
        b = {"end": prev_end + self.batch_s, "rids": rids, "done": False}
        self._batches = getattr(self, "_batches", []) + [b]
        return b

    def done(self, b):
        if not b["done"] and time.perf_counter() >= b["end"]:
            b["done"] = True
            self.inflight -= 1
        return b["done"]

    def busy(self, b):
        return self.batch_s

    def release(self, h):
        self.resident -= h["item"].bytes


def _items(sizes):
    return [Item(rid=k, n=n, params=None, bytes=100 * n, pairs=n) for k, n in enumerate(sizes)]


def test_all_served_within_budget_in_arrival_order():
    rng = np.random.default_rng(3)
    sizes = rng.integers(10, 100, 40)
    items = _items(sizes)
    arrivals = np.sort(rng.uniform(0, 0.03, 40))
    be = FakeBackend(batch_s=0.001)
    budget = 100 * 250
    st = run_policy(items, arrivals, be, budget, max_batch=8, max_inflight=2)
    assert np.all(np.isfinite(st.done_s))
    assert np.all(st.latency_s >= 0)
    assert be.max_resident <= budget and st.peak_bytes <= budget
    assert be.max_inflight <= 2
    assert max(st.batches) <= 8 and sum(st.batches) == 40
    admitted = [e[2] for e in be.events if e[0] == "admit"]
    assert admitted == sorted(admitted, key=lambda k: arrivals[k])
    assert be.resident == 0


def test_requests_arriving_during_a_batch_join_the_next_one():
    # one request at t=0, ten more while its (slow) batch runs
    items = _items([10] * 11)
    arrivals = np.array([0.0] + [0.002 + 0.0005 * k for k in range(10)])
    be = FakeBackend(batch_s=0.02)
    st = run_policy(items, arrivals, be, budget_bytes=10 ** 9, max_batch=32, max_inflight=1)
    launches = [e[2] for e in be.events if e[0] == "launch"]
    assert launches[0] == [0]
    assert launches[1] == list(range(1, 11))      # all ten in one batch
    assert st.batches == [1, 10]


def test_budget_limits_what_is_resident():
    items = _items([100] * 6)                      # 10,000 bytes each
    arrivals = np.zeros(6)
    be = FakeBackend(batch_s=0.002)
    st = run_policy(items, arrivals, be, budget_bytes=25_000, max_batch=32, max_inflight=2)
    assert be.max_resident <= 25_000
    assert max(st.batches) <= 2
    assert np.all(np.isfinite(st.done_s))


def test_request_larger_than_budget_is_refused():
    items = _items([10, 1000])
    with pytest.raises(ValueError):
        run_policy(items, np.zeros(2), FakeBackend(), budget_bytes=50_000)


def test_invalid_request_fails_alone():
    """A request the library rejects at admission is reported as failed at once; the
    others are served."""
    items = _items([10, 20, 30, 40])
    items[2].valid = False
    be = FakeBackend(batch_s=0.001)
    st = run_policy(items, np.zeros(4), be, budget_bytes=10 ** 6, max_batch=8)
    assert st.failed == [2]
    launched = [r for e in be.events if e[0] == "launch" for r in e[2]]
    assert sorted(launched) == [0, 1, 3]
    assert np.all(np.isfinite(st.done_s))


class _Ring:
    """The DeviceRing placement logic on a host stand-in for the device buffer."""

    def __new__(cls, capacity):
        from paper_1611_04474_amd import serving as S
        r = object.__new__(S.DeviceRing)
        r.capacity = S._align(capacity)
        r.base = 0
        r.live = __import__("collections").deque()
        return r


def test_device_ring_fifo_placement():
    """Slots placed in admission order and freed in launch order never overlap and always
    fit while the bytes held stay within capacity - largest slot."""
    rng = np.random.default_rng(4)
    big = 256 * 40
    ring = _Ring(256 * 400 + big)
    live = []                       # (start, size) in placement order
    held = 0
    for step in range(3000):
        if live and (rng.random() < 0.45 or held > 256 * 350):
            start, size = live.pop(0)
            ring.free(start)
            held -= size
            continue
        size = 256 * int(rng.integers(1, 41))
        if held + size > 256 * 400:
            continue
        start = ring.alloc(size)
        assert start is not None, (step, held, size)
        for s0, n0 in live:
            assert start + size <= s0 or s0 + n0 <= start
        assert 0 <= start and start + size <= ring.capacity
        live.append((start, size))
        held += size
    for start, _ in live:
        ring.free(start)
    assert not ring.live
