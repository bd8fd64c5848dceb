"""Scheduler of the render server (no GPU): admission by tile-buffer memory,
batching, retries on pair-buffer overflow, and completion of every request
even under a tiny memory pool."""
from __future__ import annotations

import types

from paper_2605_13794_amd.serve import PAIR_BYTES, Request, Scheduler, percentile, serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t


class FakeExecutor:
    """Completes a batch `dur` seconds of fake time after launch; reports a
    pair count of `ppx_true` per pixel."""

    def __init__(self, clock, dur=2e-3, ppx_true=2.0):
        self.clock, self.dur, self.ppx = clock, dur, ppx_true
        self.slots = {}
        self.launches = []

    def launch(self, slot, batch, capacity):
        # a slot is relaunched only after its batch completed (or overflowed)
        assert slot not in self.slots or self.clock.t >= self.slots[slot][0]
        self.slots[slot] = (self.clock.t + self.dur, batch, capacity)
        self.launches.append((slot, [r.rid for r in batch], capacity))

    def done(self, slot):
        return self.clock.t >= self.slots[slot][0]

    def pairs(self, slot):
        return int(sum(r.pixels for r in self.slots[slot][1]) * self.ppx)

    def capacity(self, slot):
        return self.slots[slot][2]

    def images(self, slot):
        _, batch, _ = self.slots.pop(slot)
        return [(None,)] * len(batch)


def _cam(w, h):
    return types.SimpleNamespace(width=w, height=h)


def _reqs(n, gap=1e-3):
    res = [(640, 360), (1280, 720), (1920, 1080), (3840, 2160)]
    return [Request(rid=i, arrival=i * gap, cam=_cam(*res[i % 4])) for i in range(n)]


def test_all_complete_and_memory_bounded():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(n_slots=3, max_batch=4, memory_budget=2_000_000_000, pairs_per_px=2.5)
    done, _ = serve(_reqs(60), ex, sch, clock=clock)
    assert len(done) == 60
    assert all(r.t_done >= r.arrival for r in done)
    assert sch.max_in_use <= sch.budget
    assert all(len(b) <= 4 for _, b, _ in ex.launches)
    assert sch.in_use == 0 and sorted(sch.free_slots) == [0, 1, 2]


def test_tiny_pool_queues_instead_of_failing():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    big = _cam(3840, 2160).width * _cam(3840, 2160).height
    sch = Scheduler(n_slots=4, max_batch=8, memory_budget=big * 8, pairs_per_px=2.5)
    done, _ = serve(_reqs(20, gap=1e-5), ex, sch, clock=clock)
    assert len(done) == 20
    # a 4K request alone exceeds the pool: it must have run alone
    for _, rids, _ in ex.launches:
        if any(rid % 4 == 3 for rid in rids):
            assert len(rids) == 1


def test_overflow_is_retried_with_a_larger_estimate():
    clock = FakeClock()
    ex = FakeExecutor(clock, ppx_true=9.0)
    sch = Scheduler(n_slots=2, max_batch=2, memory_budget=10**12, pairs_per_px=1.0)
    done, _ = serve(_reqs(8), ex, sch, clock=clock)
    assert len(done) == 8
    assert any(r.retries > 0 for r in done)
    assert sch.ppx >= 9.0
    # every completed launch had room for its pairs
    assert all(r.pairs <= max(c for _, ids, c in ex.launches if r.rid in ids) for r in done)


def test_overflow_beyond_the_largest_buffer_raises():
    """An executor whose buffers cannot grow past a cap: the server gives up
    after its retries instead of re-queueing forever."""
    import pytest

    class Capped(FakeExecutor):
        def launch(self, slot, batch, capacity):
            super().launch(slot, batch, min(capacity, 1000))

    clock = FakeClock()
    ex = Capped(clock, ppx_true=2.0)
    sch = Scheduler(n_slots=1, max_batch=1, memory_budget=10**12, pairs_per_px=1.0)
    with pytest.raises(RuntimeError, match="after 3 retries"):
        serve(_reqs(2), ex, sch, clock=clock, max_retries=3)


def test_fifo_start_order():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(n_slots=1, max_batch=1, memory_budget=10**12)
    done, _ = serve(_reqs(10), ex, sch, clock=clock)
    starts = [r.rid for r in sorted(done, key=lambda r: r.t_start)]
    assert starts == list(range(10))


def test_charge_scales_with_pixels():
    sch = Scheduler(1, 1, 10**12, pairs_per_px=2.0, margin=1.0)
    r1 = Request(0, 0.0, _cam(640, 360))
    r2 = Request(1, 0.0, _cam(1280, 720))
    assert sch.charge(r2) == 4 * sch.charge(r1)
    assert sch.charge(r1) == 640 * 360 * (2 * PAIR_BYTES + 20)


def test_percentile():
    assert percentile([1, 2, 3, 4, 5], 50) == 3
    assert abs(percentile(list(range(101)), 99) - 99) < 1e-9


class DeviceClockExecutor(FakeExecutor):
    """Like FakeExecutor, but keeps device time stamps: a batch completes on
    the device `dur` after its launch, while the host observes it later."""

    def start_clock(self):
        self.ref = self.clock.t

    def device_time(self, slot):
        return self.slots[slot][0] - self.ref


def test_latency_uses_device_completion_time():
    clock = FakeClock()
    ex = DeviceClockExecutor(clock, dur=2e-3)
    sch = Scheduler(n_slots=2, max_batch=4, memory_budget=1 << 40)
    done, _ = serve(_reqs(20), ex, sch, clock=clock)
    assert len(done) == 20
    for r in done:
        # completion on the device clock, never after the host saw it
        assert r.t_done is not None and r.t_seen is not None
        assert r.arrival <= r.t_done <= r.t_seen + 1e-12
