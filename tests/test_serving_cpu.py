"""Host logic of the continuous-batching server, with a simulated device.

The fake backend gives every request a service time proportional to its
footprint and runs admitted requests concurrently on a virtual clock, so the
tests check the admission rules exactly: a request starts only after it
arrives, never more than `slots` run at once, the running footprints never
exceed the budget, arrival order is kept except where the look-ahead lets a
request that fits pass one that does not, and an oversized request is
rejected before anything runs.
"""
import numpy as np
import pytest

from paper_2303_11612_amd.serving import (Request, Server, percentile, poisson_arrivals,
                                          summarize)


class _FakeTensor:
    def __init__(self, nbytes):
        self.nbytes = nbytes


class FakeBackend:
    def __init__(self, rate=1e9, dt=1e-5):
        self.now = 0.0
        self.rate = rate            # bytes per second of service
        self.dt = dt
        self.running = {}           # rid -> (start, end, footprint)
        self.log = []               # (time, event, rid, running footprints, running count)

    def footprint(self, req):
        return req.X.nbytes

    def reference(self):
        return None, 0.0

    def clock(self):
        return self.now

    def idle(self):
        self.now += self.dt

    def launch(self, req, slot):
        end = self.now + req.X.nbytes / self.rate
        self.running[req.rid] = (self.now, end, req.X.nbytes)
        self.log.append((self.now, "start", req.rid, sum(v[2] for v in self.running.values()),
                         len(self.running)))
        return req.rid

    def poll(self, h):
        return self.now >= self.running[h][1]

    def completion_time(self, h, ref):
        return self.running[h][1]

    def finish(self, h, res):
        self.running.pop(h)
        self.log.append((self.now, "end", h, 0, len(self.running)))


def _reqs(sizes, arrivals):
    return [Request(i, _FakeTensor(int(s)), (4, 4, 4), arrival=float(a))
            for i, (s, a) in enumerate(zip(sizes, arrivals))]


def _serve(reqs, slots, budget, lookahead=8, **kw):
    be = FakeBackend(**kw)
    srv = Server(be, slots=slots, hbm_budget=budget, lookahead=lookahead)
    res = srv.run(reqs, clock=be.clock, idle=be.idle)
    return be, srv, res


def test_slots_budget_and_arrivals_respected():
    rng = np.random.default_rng(0)
    sizes = rng.integers(1 << 20, 64 << 20, size=60)
    arr = poisson_arrivals(60, 2000.0, seed=1)
    reqs = _reqs(sizes, arr)
    budget = 128 << 20
    be, srv, res = _serve(reqs, slots=3, budget=budget)
    assert [r.rid for r in res] == list(range(60))
    for t, ev, rid, used, n in be.log:
        if ev == "start":
            assert used <= budget
            assert n <= 3
            assert t >= reqs[rid].arrival
    assert srv.peak_used <= budget
    for r in res:
        assert r.admitted >= r.arrival
        assert r.completed > r.admitted
        assert r.latency > 0


def test_one_slot_is_fifo():
    sizes = [8 << 20, 1 << 20, 4 << 20, 2 << 20]
    be, _, res = _serve(_reqs(sizes, [0.0, 1e-6, 2e-6, 3e-6]), slots=1, budget=1 << 30)
    starts = [rid for _, ev, rid, _, _ in be.log if ev == "start"]
    assert starts == [0, 1, 2, 3]
    # back to back: each starts when the previous ends
    for a, b in zip(res, res[1:]):
        assert b.admitted >= a.completed - 1e-12


def test_lookahead_lets_small_request_pass_large_one():
    # budget fits the running 60 MB request plus a 30 MB one, not a 70 MB one
    MB = 1 << 20
    sizes = [60 * MB, 70 * MB, 30 * MB]
    be, _, res = _serve(_reqs(sizes, [0.0, 1e-6, 2e-6]), slots=4, budget=100 * MB)
    starts = [rid for _, ev, rid, _, _ in be.log if ev == "start"]
    assert starts == [0, 2, 1]
    assert res[2].admitted < res[1].admitted
    # the large one starts only once enough has completed
    assert res[1].admitted >= min(res[0].completed, res[2].completed)


def test_lookahead_one_keeps_strict_order():
    MB = 1 << 20
    sizes = [60 * MB, 70 * MB, 30 * MB]
    be, _, _ = _serve(_reqs(sizes, [0.0, 1e-6, 2e-6]), slots=4, budget=100 * MB, lookahead=1)
    starts = [rid for _, ev, rid, _, _ in be.log if ev == "start"]
    assert starts == [0, 1, 2]


def test_request_larger_than_budget_rejected():
    with pytest.raises(ValueError, match="budget"):
        _serve(_reqs([10, 200], [0.0, 0.0]), slots=2, budget=100)


def test_concurrency_lowers_latency_under_load():
    # at 70% of the one-slot capacity, several slots shorten the queue
    rng = np.random.default_rng(3)
    sizes = rng.integers(1 << 20, 32 << 20, size=200)
    rate_b = 4e9
    mean_service = float(np.mean(sizes)) / rate_b
    arr = poisson_arrivals(200, 0.7 / mean_service, seed=4)
    _, _, one = _serve(_reqs(sizes, arr), slots=1, budget=1 << 34, rate=rate_b)
    _, _, many = _serve(_reqs(sizes, arr), slots=4, budget=1 << 34, rate=rate_b)
    s1, s4 = summarize(one), summarize(many)
    assert s4["p99_ms"] < s1["p99_ms"]
    assert s4["p50_ms"] <= s1["p50_ms"]


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50
    assert percentile(xs, 99) == 99
    assert percentile(xs, 100) == 100
    assert percentile([5.0], 99) == 5.0
    assert np.isnan(percentile([], 50))


def test_poisson_arrivals_rate():
    a = poisson_arrivals(20000, 500.0, seed=0)
    assert np.all(np.diff(a) > 0)
    assert abs(20000 / a[-1] - 500.0) < 15.0


class FakeGroupedBackend(FakeBackend):
    """A group costs a fixed launch overhead plus its bytes at the service
    rate (the grouped kernels pay the per-stage launch cost once per group)."""

    grouped = True

    def __init__(self, max_group=4, overhead=2e-3, **kw):
        super().__init__(**kw)
        self.max_group = max_group
        self.overhead = overhead
        self.groups = []

    def compatible(self, a, b):
        return len(a.ranks) == len(b.ranks)

    def launch_group(self, reqs, slot):
        nbytes = sum(r.X.nbytes for r in reqs)
        end = self.now + self.overhead + nbytes / self.rate
        key = tuple(r.rid for r in reqs)
        self.running[key] = (self.now, end, nbytes)
        self.groups.append((self.now, key))
        self.log.append((self.now, "start", key, sum(v[2] for v in self.running.values()),
                         len(self.running)))
        return key

    def finish_group(self, h, results):
        self.running.pop(h)
        self.log.append((self.now, "end", h, 0, len(self.running)))


def test_grouped_admission_rules():
    rng = np.random.default_rng(5)
    sizes = rng.integers(1 << 20, 16 << 20, size=80)
    arr = poisson_arrivals(80, 3000.0, seed=6)
    reqs = _reqs(sizes, arr)
    budget = 96 << 20
    be = FakeGroupedBackend(max_group=5)
    srv = Server(be, slots=2, hbm_budget=budget)
    res = srv.run(reqs, clock=be.clock, idle=be.idle)
    assert [r.rid for r in res] == list(range(80))
    seen = []
    for t, key in be.groups:
        assert 1 <= len(key) <= 5
        assert all(reqs[rid].arrival <= t for rid in key)
        seen += list(key)
    assert sorted(seen) == list(range(80))
    assert sum(srv.group_sizes) == 80 and max(srv.group_sizes) > 1
    for t, ev, key, used, n in be.log:
        if ev == "start":
            assert used <= budget and n <= 2
    # members of a group complete together
    for _, key in be.groups:
        assert len({res[rid].completed for rid in key}) == 1


def test_grouping_amortises_launch_overhead_under_load():
    sizes = np.full(120, 1 << 20)
    arr = poisson_arrivals(120, 1500.0, seed=8)      # 1.5x what one-at-a-time sustains
    def run(gmax):
        be = FakeGroupedBackend(max_group=gmax, overhead=1e-3, rate=1e12)
        return summarize(Server(be, slots=1, hbm_budget=1 << 34).run(
            _reqs(sizes, arr), clock=be.clock, idle=be.idle))
    one, grouped = run(1), run(32)
    assert grouped["throughput_rps"] > 1.3 * one["throughput_rps"]
    assert grouped["p99_ms"] < one["p99_ms"]
