"""Scheduling logic of the continuous-batching request loop, on the CPU with a
fake pool: footprint admission in arrival order, joining a running set,
completion accounting, slot and memory reuse, idle waiting."""
import pytest

from paper_1810_07802_amd import serve


class FakePool:
    """Pool with the HIP pool's interface: a byte budget and a slot table;
    one step of the running set costs `cost` seconds of simulated time per
    running case, advanced on `clock`."""

    def __init__(self, budget, max_cases, clock, cost=1e-3, poison=()):
        self.budget, self.max_cases, self.clock, self.cost = budget, max_cases, clock, cost
        self.poison = set(poison)  # rids whose state goes non-finite at their first step
        self.bad = set()           # slots whose state is non-finite
        self.used = 0
        self.slots = {}  # slot -> [remaining, bytes, done]
        self.admit_log, self.step_log = [], []

    def admit(self, case, steps):
        b = case["nx"] * case["ny"] * 168
        free = [k for k in range(self.max_cases) if k not in self.slots]
        if not free or self.used + b > self.budget:
            return None
        k = free[0]
        self.slots[k] = [steps, b, 0]
        self.rid_of = getattr(self, "rid_of", {})
        self.rid_of[k] = case["rid"]
        self.used += b
        self.admit_log.append((case["rid"], self.clock.t))
        return k

    def step(self, n, use_graph=True):
        running = [s for s in self.slots.values() if s[0] > 0]
        self.step_log.append(len(running))
        for k, s in self.slots.items():
            if s[0] > 0 and self.rid_of[k] in self.poison:
                self.bad.add(k)
        for s in running:
            d = min(n, s[0])
            s[0] -= d
            s[2] += d
        self.clock.t += n * self.cost * max(1, len(running))

    def remaining(self, k):
        return self.slots[k][0]

    def status(self, k):
        return -4 if k in self.bad else 0

    def macros(self, k):
        return {"done": self.slots[k][2]}

    def retire(self, k):
        self.used -= self.slots.pop(k)[1]
        self.bad.discard(k)

    def sync(self):
        pass


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def req(rid, n, steps, arrival):
    return serve.Request(rid, {"rid": rid, "nx": n, "ny": n}, steps, arrival)


def test_every_request_completes_with_its_own_step_count():
    clk = Clock()
    pool = FakePool(budget=10**9, max_cases=8, clock=clk)
    reqs = [req(k, 16 * (k + 1), 50 * (k + 1), 0.0) for k in range(5)]
    out = serve.run(pool, reqs, chunk=20, clock=clk, sleep=clk.sleep)
    assert sorted(s.rid for s in out) == list(range(5))
    for s in out:
        assert s.macros["done"] == s.steps  # a case stops at its own target
        assert s.finished >= s.admitted >= s.arrival
    # shorter requests finish first when all start together
    assert [s.rid for s in out] == sorted(s.rid for s in out)
    assert not pool.slots and pool.used == 0


def test_arrivals_join_the_running_set():
    clk = Clock()
    pool = FakePool(budget=10**9, max_cases=8, clock=clk)
    reqs = [req(0, 32, 1000, 0.0), req(1, 32, 100, 0.05)]
    out = serve.run(pool, reqs, chunk=10, clock=clk, sleep=clk.sleep)
    first = {s.rid: s for s in out}
    # request 1 is admitted while request 0 runs and finishes before it
    assert first[1].admitted < first[0].finished
    assert out[0].rid == 1
    assert max(pool.step_log) == 2


def test_footprint_admission_waits_for_memory_in_arrival_order():
    clk = Clock()
    big = 64 * 64 * 168
    pool = FakePool(budget=2 * big, max_cases=8, clock=clk)
    reqs = [req(0, 64, 100, 0.0), req(1, 64, 300, 0.0), req(2, 64, 50, 0.0), req(3, 16, 10, 0.0)]
    out = serve.run(pool, reqs, chunk=10, clock=clk, sleep=clk.sleep)
    by = {s.rid: s for s in out}
    # only two fit at once: request 2 waits for request 0's memory, and request
    # 3 (small, would fit) still waits behind it: arrival order is kept
    assert by[2].admitted >= by[0].finished
    assert [r for r, _ in pool.admit_log] == [0, 1, 2, 3]
    assert pool.used == 0


def test_slot_limit_is_respected():
    clk = Clock()
    pool = FakePool(budget=10**12, max_cases=2, clock=clk)
    reqs = [req(k, 8, 20, 0.0) for k in range(6)]
    out = serve.run(pool, reqs, chunk=5, clock=clk, sleep=clk.sleep)
    assert len(out) == 6 and max(pool.step_log) <= 2


def test_idle_pool_sleeps_until_the_next_arrival():
    clk = Clock()
    pool = FakePool(budget=10**9, max_cases=4, clock=clk, cost=1e-4)
    reqs = [req(0, 8, 10, 1.0), req(1, 8, 10, 5.0)]
    out = serve.run(pool, reqs, chunk=10, clock=clk, sleep=clk.sleep)
    by = {s.rid: s for s in out}
    assert by[0].admitted == pytest.approx(1.0) and by[1].admitted == pytest.approx(5.0)
    assert by[1].tts == pytest.approx(10 * 1e-4)


def test_a_request_larger_than_the_empty_pool_is_an_error():
    clk = Clock()
    pool = FakePool(budget=1000, max_cases=4, clock=clk)
    with pytest.raises(RuntimeError):
        serve.run(pool, [req(0, 64, 10, 0.0)], clock=clk, sleep=clk.sleep)


def test_summary_percentiles():
    s = [serve.Served(k, 100, 10, 0.0, 0.0, float(k + 1)) for k in range(100)]
    m = serve.summary(s)
    assert m["p50_s"] == pytest.approx(50.5) and m["p99_s"] == pytest.approx(99.01)
    assert m["mlups"] == pytest.approx(100 * 100 * 10 / 100.0 / 1e6)


def test_a_request_that_goes_non_finite_fails_alone_and_frees_its_slot():
    """The pool reports ENUMERIC for one slot (its state went non-finite):
    that request is retired with an error at the next look, its slot and
    memory are reused, and every other request completes with its result."""
    clk = Clock()
    pool = FakePool(budget=3 * 64 * 64 * 168, max_cases=2, clock=clk, poison={1})
    reqs = [req(k, 64, 100, 0.0) for k in range(5)]
    out = serve.run(pool, reqs, chunk=20, clock=clk, sleep=clk.sleep)
    by = {s.rid: s for s in out}
    assert sorted(by) == list(range(5))
    assert by[1].error == "ENUMERIC" and by[1].macros is None
    # failed at the first look, long before its 100 steps
    assert by[1].finished - by[1].admitted <= 20 * pool.cost * 2 + 1e-12
    for k in (0, 2, 3, 4):
        assert by[k].error is None and by[k].macros["done"] == 100
    assert not pool.slots and pool.used == 0
    summ = serve.summary(out)
    assert summ["failed"] == 1 and summ["requests"] == 5
