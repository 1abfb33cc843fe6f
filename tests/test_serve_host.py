"""The serving loop's scheduling on the CPU, with a simulated executor and clock.

The simulated executor finishes a launch after a time proportional to its
effective flops; the checks are on admission (arrival order, HBM budget,
slots), continuous batching and the latency accounting.
"""

import numpy as np
import pytest

from paper_1905_07439_amd import serve


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def advance_to(self, t):
        assert t >= self.t
        self.t = t


class FakeExecutor:
    def __init__(self, clock, scheduler, rate=1e12, overhead=1e-4):
        self.clock, self.scheduler, self.rate, self.overhead = clock, scheduler, rate, overhead
        self.launches = []
        self.running = 0
        self.max_running = 0

    def footprint(self, r):
        return 3 * r.n * r.n * 4

    def start(self, t0):
        pass

    def launch(self, reqs, slot):
        assert self.scheduler.in_use <= self.scheduler.budget
        done = self.clock.now() + self.overhead + sum(2.0 * r.n ** 3 for r in reqs) / self.rate
        h = {"done": done, "reqs": list(reqs), "slot": slot}
        self.launches.append(h)
        self.running += 1
        self.max_running = max(self.max_running, self.running)
        return h

    def poll(self, h):
        return h["done"] if self.clock.now() >= h["done"] else None

    def next_done(self, h):
        return h["done"]

    def finish(self, h):
        self.running -= 1

    def stop(self):
        pass


def _run(reqs, budget=1 << 40, slots=4, max_batch=64, rate=1e12):
    clock = SimClock()
    sch = serve.Scheduler(budget, max_batch)
    ex = FakeExecutor(clock, sch, rate)
    stats = serve.serve(reqs, ex, sch, slots=slots, clock=clock)
    return stats, ex, sch


def test_requests_follow_the_configured_mix():
    reqs = serve.make_requests(2000, 1.0, 7)
    assert 1800 < len(reqs) < 2200
    n = np.array([r.n for r in reqs])
    assert n.min() >= 128 and n.max() <= 4096 and (n % 32 == 0).all()
    # log-uniform: the median is near the geometric mean sqrt(128 * 4096) = 724
    assert 600 < np.median(n) < 880
    counts = {s: sum(r.scheme == s for r in reqs) for s in serve.SCHEMES}
    assert all(550 < c < 800 for c in counts.values())
    assert [r.seed for r in reqs] == list(range(len(reqs)))


def test_levels_give_leaves_of_about_96_to_256():
    for n in range(128, 4097, 32):
        for s in serve.SCHEMES:
            q = len(serve.levels_for(n, s))
            leaf = n / (3 if s == "laderman" else 2) ** q
            assert q >= 1 and (leaf <= 340 or q == 1), (n, s, q)
            assert leaf >= 42, (n, s, q)


def test_all_requests_complete_in_arrival_order_of_admission():
    reqs = serve.make_requests(2000, 0.2, 3, hi=1024)
    stats, ex, _ = _run(reqs)
    assert stats["requests"] == len(reqs)
    adm = [r.admitted for r in sorted(reqs, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    for r in reqs:
        assert r.arrival <= r.admitted <= r.done
    assert sum(len(h["reqs"]) for h in ex.launches) == len(reqs)


def test_budget_limits_what_is_in_flight():
    reqs = serve.make_requests(4000, 0.1, 5, lo=512, hi=2048)
    biggest = max(3 * r.n * r.n * 4 for r in reqs)
    stats, ex, sch = _run(reqs, budget=2 * biggest, rate=2e10)
    assert sch.peak <= 2 * biggest and sch.in_use == 0
    with pytest.raises(ValueError):
        _run(reqs, budget=biggest // 2)


def test_continuous_batching_admits_arrivals_when_a_slot_frees():
    # One slot, a long first request: everything arriving meanwhile is launched together
    # as soon as it completes.
    R = serve.Request
    reqs = [R(0, 0.0, 4096, "strassen", 0)] + [R(i, 0.001 * i, 256, "strassen", i) for i in range(1, 6)]
    stats, ex, _ = _run(reqs, slots=1, rate=1e12)
    first = ex.launches[0]
    assert [r.rid for r in first["reqs"]] == [0]
    assert [r.rid for r in ex.launches[1]["reqs"]] == [1, 2, 3, 4, 5]
    assert all(r.admitted == pytest.approx(first["done"]) for r in reqs[1:])
    # with more slots they run beside it
    one_slot = [r.done - r.arrival for r in reqs[1:]]
    stats4, ex4, _ = _run(reqs, slots=4, rate=1e12)
    assert ex4.max_running >= 2
    assert max(r.done - r.arrival for r in reqs[1:]) < min(one_slot)


def test_latency_statistics():
    R = serve.Request
    reqs = [R(i, 0.01 * i, 1000, "strassen", i) for i in range(10)]
    stats, ex, _ = _run(reqs, rate=2e12, slots=1)
    # each request alone: 2e9 / 2e12 = 1 ms plus 0.1 ms overhead, no queueing
    assert stats["latency_ms"]["p50"] == pytest.approx(1.1)
    assert stats["latency_ms"]["max"] == pytest.approx(1.1)
    assert stats["batches"] == 10 and stats["mean_batch"] == 1.0
