"""Scheduler logic of the continuous-batching loop, on the CPU with a fake
executor and a fake clock (no GPU): admission by HBM footprint, FIFO order per
parameter set, batching of requests that arrive while others run, rejection
of requests that can never fit, and the latency statistics."""
import pytest

from paper_2603_16692_amd.serving import (Executor, Request, Scheduler, choose_sets, latency_stats,
                                          poisson_offsets)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    """Service time = base + per_item * batch on the fake clock; result = 3 * payload + set offset."""

    def __init__(self, clock, per_item_bytes, resident=0, base=1e-3, per_item=2e-4):
        self.clock, self.per_item_bytes, self.resident = clock, per_item_bytes, resident
        self.base, self.per_item = base, per_item
        self.launched = []

    def resident_bytes(self):
        return self.resident

    def footprint(self, set_name, batch):
        return self.per_item_bytes[set_name] * batch

    def launch(self, set_name, requests):
        end = self.clock() + self.base + self.per_item * len(requests)
        self.launched.append((set_name, [r.rid for r in requests]))
        return (end, set_name, [r.payload for r in requests])

    def poll(self, handle):
        return self.clock() >= handle[0]

    def finish(self, handle):
        off = {"a": 1, "b": 2}[handle[1]]
        return [3 * p + off for p in handle[2]]


def drive(sched, clock, reqs, offsets, dt=1e-4, limit=100000):
    order = sorted(range(len(reqs)), key=lambda i: offsets[i])
    nxt, steps = 0, 0
    while (nxt < len(order) or sched.pending()) and steps < limit:
        while nxt < len(order) and offsets[order[nxt]] <= clock.t:
            r = reqs[order[nxt]]
            r.arrival = offsets[order[nxt]]
            sched.submit(r)
            nxt += 1
        sched.step()
        clock.t += dt
        steps += 1
    assert steps < limit


def make(n, rate=2000.0, seed=3):
    names = choose_sets(n, ["a", "b"], [0.6, 0.4], seed=seed)
    offs = poisson_offsets(n, rate, seed=seed)
    return [Request(i, names[i], i) for i in range(n)], offs


def test_results_and_budget():
    clock = FakeClock()
    ex = FakeExecutor(clock, {"a": 100, "b": 250}, resident=1000)
    sched = Scheduler(ex, hbm_budget=1000 + 1500, max_batch={"a": 8, "b": 4}, slots=2, clock=clock)
    reqs, offs = make(400)
    drive(sched, clock, reqs, offs)
    assert len(sched.completed) == 400 and not sched.rejected
    for r in reqs:
        assert r.result == 3 * r.payload + {"a": 1, "b": 2}[r.set_name]
    assert sched.peak_in_use <= sched.budget
    assert sched.in_use == ex.resident_bytes()


def test_results_can_be_dropped_on_completion():
    # a long request stream keeps no outputs alive; latencies are still recorded
    clock = FakeClock()
    ex = FakeExecutor(clock, {"a": 100, "b": 250})
    sched = Scheduler(ex, hbm_budget=10000, max_batch={"a": 8, "b": 4}, slots=2, clock=clock, keep_results=False)
    reqs, offs = make(200)
    drive(sched, clock, reqs, offs)
    assert len(sched.completed) == 200
    assert all(r.result is None and r.latency is not None and r.latency > 0 for r in reqs)


def test_fifo_within_each_set_and_batching():
    clock = FakeClock()
    ex = FakeExecutor(clock, {"a": 10, "b": 10})
    sched = Scheduler(ex, hbm_budget=10 ** 9, max_batch={"a": 8, "b": 8}, slots=1, clock=clock)
    reqs, offs = make(300, rate=20000.0)  # arrivals much faster than service: queues build up
    drive(sched, clock, reqs, offs)
    for name in ("a", "b"):
        launched = [rid for s, rids in ex.launched if s == name for rid in rids]
        arrivals = sorted((r.arrival, r.rid) for r in reqs if r.set_name == name)
        assert launched == [rid for _, rid in arrivals]
    sizes = [len(rids) for _, rids in ex.launched]
    assert max(sizes) == 8 and sum(sizes) == 300
    assert all(r.admitted >= r.arrival for r in reqs)


def test_admission_waits_for_memory():
    clock = FakeClock()
    ex = FakeExecutor(clock, {"a": 100, "b": 100})
    # room for 3 items in flight in total, 4 slots
    sched = Scheduler(ex, hbm_budget=300, max_batch={"a": 8, "b": 8}, slots=4, clock=clock)
    reqs, offs = make(200, rate=50000.0)
    drive(sched, clock, reqs, offs)
    assert sched.peak_in_use <= 300
    assert all(len(rids) <= 3 for _, rids in ex.launched)
    assert len(sched.completed) == 200


def test_rejects_requests_that_never_fit():
    clock = FakeClock()
    ex = FakeExecutor(clock, {"a": 100, "b": 5000}, resident=100)
    sched = Scheduler(ex, hbm_budget=1000, max_batch={"a": 4, "b": 4}, clock=clock)
    assert sched.submit(Request(0, "a", 1))
    assert not sched.submit(Request(1, "b", 1))
    assert [r.rid for r in sched.rejected] == [1]
    with pytest.raises(KeyError):
        sched.submit(Request(2, "zzz", 1))


def test_unbatched_plain_dispatch_is_the_baseline():
    clock = FakeClock()
    ex = FakeExecutor(clock, {"a": 1, "b": 1})
    sched = Scheduler(ex, hbm_budget=10 ** 9, max_batch={"a": 1, "b": 1}, slots=1, clock=clock)
    reqs, offs = make(100, rate=20000.0)
    drive(sched, clock, reqs, offs)
    assert all(len(rids) == 1 for _, rids in ex.launched)
    # FIFO across sets when unbatched: launch order = arrival order
    order = [rids[0] for _, rids in ex.launched]
    assert order == [r.rid for r in sorted(reqs, key=lambda r: r.arrival)]


def test_batching_lowers_tail_latency_under_load():
    def p99(max_b):
        clock = FakeClock()
        ex = FakeExecutor(clock, {"a": 1, "b": 1}, base=1e-3, per_item=1e-4)
        sched = Scheduler(ex, 10 ** 9, {"a": max_b, "b": max_b}, slots=1, clock=clock)
        reqs, offs = make(300, rate=1500.0)  # above the unbatched capacity (~900/s)
        drive(sched, clock, reqs, offs, dt=5e-5)
        return latency_stats(sched.completed)["p99_ms"]
    assert p99(8) < p99(1)


def test_latency_stats_and_arrivals():
    reqs = []
    for i in range(100):
        r = Request(i, "a", 0, arrival=0.0)
        r.done = (i + 1) * 1e-3
        reqs.append(r)
    st = latency_stats(reqs)
    assert st["count"] == 100
    assert abs(st["p50_ms"] - 50.0) < 1e-9 and abs(st["p99_ms"] - 99.0) < 1e-9
    offs = poisson_offsets(20000, 1000.0, seed=1)
    assert offs == sorted(offs) and offs == poisson_offsets(20000, 1000.0, seed=1)
    assert abs(20000 / offs[-1] - 1000.0) < 30.0  # mean rate
    names = choose_sets(10000, ["a", "b", "c", "d"], [0.4, 0.3, 0.2, 0.1], seed=5)
    frac = names.count("a") / len(names)
    assert abs(frac - 0.4) < 0.02
