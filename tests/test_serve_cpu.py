"""The continuous-batching scheduler against a fake backend on the CPU:
admission by HBM footprint and free slots, FIFO blocking, slot reuse,
overlap of late arrivals with running work, and a failing slot retired with
its error while the others keep running."""
import types

import pytest

from paper_1507_07548_amd.serve import Request, Server, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Slots advance k steps per launch(k); the chunk is ready `cost` seconds
    of the fake clock later (families' chunks overlap, as on the device's
    streams).  A request whose system has `fail_at` stops there with status 4
    (non-finite)."""

    def __init__(self, clock, max_slots=4, cost=0.01, bytes_per_mol=100):
        self.clock, self.max_slots, self.cost, self.bpm = clock, max_slots, cost, bytes_per_mol
        self.slots = {}
        self.peak_active = 0
        self.admitted = []
        self.busy_until = 0.0
        self.last_status = 5

    def footprint(self, system, precision):
        return system.n * self.bpm

    def admit(self, system, precision):
        if len(self.slots) >= self.max_slots:
            return None
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = {"sys": system, "steps": 0, "status": 0}
        self.admitted.append(system.rid)
        self.peak_active = max(self.peak_active, len(self.slots))
        return slot

    def active(self):
        return len(self.slots)

    def launch(self, k):
        assert self.ready(), "a chunk was launched while the previous one was in flight"
        for s in self.slots.values():
            if s["status"] or s["steps"] >= s["sys"].md.n_steps:
                continue
            fail = getattr(s["sys"], "fail_at", None)
            new = min(s["steps"] + k, s["sys"].md.n_steps)
            if fail is not None and new >= fail:
                s["steps"], s["status"] = fail, 4
            else:
                s["steps"] = new
        self.busy_until = self.clock.t + self.cost

    def ready(self):
        return self.clock.t >= self.busy_until

    def poll(self):
        return [(slot, s["steps"], s["status"], s["status"] != 0 or s["steps"] >= s["sys"].md.n_steps)
                for slot, s in self.slots.items()]

    def collect(self, slot):
        return {"steps": self.slots[slot]["steps"]}

    def retire(self, slot):
        del self.slots[slot]


def req(rid, arrival, n=100, steps=300, model="a", fail_at=None):
    sysm = types.SimpleNamespace(n=n, md=types.SimpleNamespace(n_steps=steps), rid=rid, fail_at=fail_at)
    return Request(rid, arrival, model, sysm)


def test_all_requests_complete_with_their_own_step_budgets():
    clk = FakeClock()
    be = FakeBackend(clk)
    srv = Server({"a": be}, hbm_budget=10 ** 9, chunk_steps=100, clock=clk, sleep=clk.sleep)
    reqs = [req(i, 0.001 * i, steps=100 * (1 + i % 3)) for i in range(10)]
    res = srv.run(reqs)
    assert sorted(r.rid for r in res) == list(range(10))
    for r in res:
        assert r.status == 0 and r.steps_done == reqs[r.rid].system.md.n_steps
        assert r.finished >= r.admitted >= r.arrival


def test_admission_respects_the_hbm_budget_and_queues_in_order():
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=16)
    budget = 250 * 100                                 # 2.5 systems of n=100
    srv = Server({"a": be}, hbm_budget=budget, chunk_steps=100, clock=clk, sleep=clk.sleep)
    res = srv.run([req(i, 0.0) for i in range(6)])
    assert be.peak_active == 2                          # never more than the budget allows
    assert be.admitted == list(range(6))                # FIFO
    waits = sorted(r.admitted - r.arrival for r in res)
    assert waits[0] == 0.0 and waits[-1] > 0.0          # later requests queued


def test_slots_are_reused_and_late_arrivals_overlap_running_work():
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=3)
    srv = Server({"a": be}, hbm_budget=10 ** 9, chunk_steps=50, clock=clk, sleep=clk.sleep)
    reqs = [req(0, 0.0, steps=1000), req(1, 0.015, steps=100), req(2, 0.03, steps=100),
            req(3, 0.035, steps=100), req(4, 0.2, steps=100)]
    res = {r.rid: r for r in srv.run(reqs)}
    # requests 1-3 were admitted and finished while request 0 was still running
    assert all(res[k].admitted < res[0].finished and res[k].finished < res[0].finished for k in (1, 2, 3))
    assert len(res) == 5 and be.peak_active == 3


def test_a_failing_slot_is_retired_while_others_continue():
    clk = FakeClock()
    be = FakeBackend(clk)
    srv = Server({"a": be}, hbm_budget=10 ** 9, chunk_steps=100, clock=clk, sleep=clk.sleep)
    res = {r.rid: r for r in srv.run([req(0, 0.0, steps=500), req(1, 0.0, steps=500, fail_at=150),
                                      req(2, 0.0, steps=500)])}
    assert res[1].status == 4 and res[1].steps_done == 150
    assert res[0].status == 0 and res[0].steps_done == 500
    assert res[2].status == 0 and res[1].finished < res[0].finished


def test_two_model_families_share_the_budget():
    clk = FakeClock()
    a, b = FakeBackend(clk, max_slots=8), FakeBackend(clk, max_slots=8, cost=0.0)
    srv = Server({"a": a, "b": b}, hbm_budget=3 * 100 * 100, chunk_steps=100, clock=clk, sleep=clk.sleep)
    reqs = [req(i, 0.0, model="ab"[i % 2]) for i in range(8)]
    res = srv.run(reqs)
    assert len(res) == 8
    assert a.peak_active + b.peak_active <= 3 + 1


def test_a_request_that_can_never_fit_fails_without_blocking_the_rest():
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=4)
    srv = Server({"a": be}, hbm_budget=300 * 100, chunk_steps=100, clock=clk, sleep=clk.sleep)
    reqs = [req(0, 0.0), req(1, 0.001, n=400), req(2, 0.002), req(3, 0.003)]
    res = {r.rid: r for r in srv.run(reqs)}
    assert sorted(res) == [0, 1, 2, 3]
    assert res[1].status == 2 and res[1].steps_done == 0 and 1 not in be.admitted
    assert all(res[k].status == 0 and res[k].steps_done == 300 for k in (0, 2, 3))


def test_a_request_refused_by_an_idle_backend_fails():
    clk = FakeClock()
    full = FakeBackend(clk, max_slots=0)
    ok = FakeBackend(clk, max_slots=2)
    srv = Server({"full": full, "ok": ok}, hbm_budget=10 ** 9, chunk_steps=100, clock=clk, sleep=clk.sleep)
    res = {r.rid: r for r in srv.run([req(0, 0.0, model="full"), req(1, 0.5, model="ok")])}
    assert res[0].status == 5 and res[0].steps_done == 0
    assert res[1].status == 0 and res[1].steps_done == 300


def test_families_progress_independently():
    """A request of a fast family arriving while a slow family's chunk is on
    the device is admitted, run and finished before that chunk ends."""
    clk = FakeClock()
    slow, fast = FakeBackend(clk, cost=1.0), FakeBackend(clk, cost=0.01)
    srv = Server({"slow": slow, "fast": fast}, hbm_budget=10 ** 9, chunk_steps=100, clock=clk, sleep=clk.sleep)
    res = {r.rid: r for r in srv.run([req(0, 0.0, model="slow", steps=200), req(1, 0.1, model="fast", steps=300)])}
    assert res[1].status == 0 and res[1].finished < 1.0
    assert res[0].finished >= 2.0
    assert res[1].admitted - res[1].arrival < 0.01


def test_nearest_rank_percentiles():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0


def test_requests_join_a_batch_by_family_and_size_class():
    from paper_1507_07548_amd.serve import SIZE_CLASSES, backend_key, size_class
    small, large = SIZE_CLASSES[0], SIZE_CLASSES[-1]
    last = len(SIZE_CLASSES)
    assert backend_key("2cljq", 256) == "2cljq/0"
    assert backend_key("2cljq", small - 1) == "2cljq/0" and backend_key("2cljq", small) == "2cljq/1"
    assert backend_key("ionic", large - 1) == f"ionic/{last - 1}" and backend_key("ionic", large) == f"ionic/{last}"
    assert backend_key("lj", 8192) == f"lj/{last}"
    assert [size_class(n, (1000, 2000, 4000)) for n in (999, 1000, 1999, 2000, 3999, 4000)] == [0, 1, 1, 2, 2, 3]
    assert backend_key("lj", 3000, classes=(1000, 2000, 4000)) == "lj/2"


class SharedDevice:
    """Counts the fake families' chunks in flight on one device."""

    def __init__(self, clock):
        self.clock, self.members, self.peak = clock, [], 0

    def add(self, be):
        self.members.append(be)
        orig = be.launch

        def launch(k):
            orig(k)
            self.peak = max(self.peak, sum(not m.ready() for m in self.members))
        be.launch = launch
        return be


def test_shortest_remaining_work_goes_first_when_launches_are_limited():
    """With one family in flight at a time, a small request that arrives
    while a large batch is running takes the device at the next chunk
    boundary and completes long before the large one; the large one still
    completes."""
    clk = FakeClock()
    dev = SharedDevice(clk)
    big = dev.add(FakeBackend(clk, cost=1.0))
    small = dev.add(FakeBackend(clk, cost=0.01))
    srv = Server({"big": big, "small": small}, hbm_budget=10 ** 9, chunk_steps=100, clock=clk,
                 sleep=clk.sleep, max_inflight=1)
    res = {r.rid: r for r in srv.run([req(0, 0.0, n=4000, model="big", steps=500),
                                      req(1, 0.5, n=100, model="small", steps=300)])}
    assert dev.peak == 1
    assert res[1].status == 0 and res[1].steps_done == 300
    assert 1.0 <= res[1].finished < 1.1            # waited for one large chunk only
    assert res[0].status == 0 and res[0].steps_done == 500 and res[0].finished >= 5.0


def test_launch_order_counts_the_whole_batch_cost():
    """A family whose nearest request is short but whose batch is expensive
    per step waits behind a family that is cheaper to finish."""
    clk = FakeClock()
    dev = SharedDevice(clk)
    a = dev.add(FakeBackend(clk, max_slots=4, cost=0.1))
    b = dev.add(FakeBackend(clk, max_slots=4, cost=0.1))
    order = []
    for name, be in (("a", a), ("b", b)):
        inner = be.launch

        def launch(k, name=name, inner=inner):
            order.append(name)
            inner(k)
        be.launch = launch
    # a: nearest request 200 steps, three n=1000 systems per step (cost 2 x 3e6 = 6e6)
    # b: nearest request 400 steps, one n=500 system (cost 4 x 2.5e5 = 1e6)
    reqs = [req(0, 0.0, n=1000, model="a", steps=200), req(1, 0.0, n=1000, model="a", steps=900),
            req(2, 0.0, n=1000, model="a", steps=900), req(3, 0.0, n=500, model="b", steps=400)]
    srv = Server({"a": a, "b": b}, hbm_budget=10 ** 9, chunk_steps=100, clock=clk, sleep=clk.sleep,
                 max_inflight=1)
    res = {r.rid: r for r in srv.run(reqs)}
    assert order[:4] == ["b"] * 4 and dev.peak == 1
    assert res[3].finished < res[0].finished
    assert all(r.status == 0 for r in res.values())


def test_max_inflight_must_be_positive():
    with pytest.raises(ValueError):
        Server({}, hbm_budget=1, max_inflight=0)
