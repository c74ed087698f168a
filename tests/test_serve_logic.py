"""Host logic of the serving loop against a simulated device and clock (CPU):
admission order (first-come first-served, shortest job first), the HBM budget
and slot limits, completion at each request's own step count, latency
accounting and the refusal of a request that cannot fit."""
import numpy as np
import pytest

from paper_2009_12584_amd.serve import Request, serve, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakePool:
    """A device that runs one launch (one step of every joined slot) in
    step_time seconds of the simulated clock, back to back; a slot joins at
    the next launch after its admission, as in the library's pool."""

    instances = []

    def __init__(self, clock, step_time, bytes_per_node, budget, max_slots, **_):
        self.clock, self.step_time, self.bpn = clock, step_time, bytes_per_node
        self.budget, self.max_slots = budget, max_slots
        self.used, self.slots, self.next_id = 0, {}, 0
        self.launched, self.busy_until, self.chunks = 0, 0.0, []
        self.admitted, self.closed = [], False
        FakePool.instances.append(self)

    def admit(self, mask, rhoA0, rhoB0, nsteps, **prm):
        need = int(np.asarray(mask).size) * self.bpn
        if len(self.slots) >= self.max_slots or self.used + need > self.budget:
            return None
        s = self.next_id
        self.next_id += 1
        self.slots[s] = dict(L0=self.launched, steps=nsteps, bytes=need, done=False, tag=prm.get("tag"),
                             fail_at=prm.get("fail_at"), broken=False)
        self.used += need
        assert self.used <= self.budget
        self.admitted.append(s)
        return s

    def advance(self, chunk):
        start = max(self.clock.now(), self.busy_until)
        self.busy_until = start + chunk * self.step_time
        self.launched += chunk
        self.chunks.append((self.busy_until, self.launched))

    def completed(self):
        c = 0
        for end, n in self.chunks:
            if end <= self.clock.now():
                c = n
        return c

    def progress(self):
        return self.launched, self.completed()

    def poll(self, max_n=256):
        c = self.completed()
        out = []
        for s, v in self.slots.items():
            if v["done"]:
                continue
            if v["fail_at"] is not None and v["L0"] + v["fail_at"] <= c:
                # the library reports a slot its diagnostics flagged, and stops it
                v["done"] = v["broken"] = True
                out.append(s)
            elif v["L0"] + v["steps"] <= c:
                v["done"] = True
                out.append(s)
        return out[:max_n]

    def status(self, slot):
        return -5 if self.slots[slot]["broken"] else 0

    def fields(self, slot, raise_on_flags=True):
        return None

    def release(self, slot):
        self.used -= self.slots.pop(slot)["bytes"]

    def close(self):
        self.closed = True


def make_requests(specs):
    """specs: (arrival s, nx, ny, steps, tag)."""
    out = []
    for t, nx, ny, steps, tag in specs:
        m = np.zeros((ny, nx), np.uint8)
        out.append(Request(t, m, None, None, steps, {}, tag=tag))
    return out


def run(reqs, clock, *, budget=10**9, slots=64, step_time=1e-4, chunk=10, policy="fifo", time_scale=1.0):
    FakePool.instances.clear()
    factory = lambda b, n, **kw: FakePool(clock, step_time, 1, b, n)
    done, makespan = serve(reqs, hbm_budget=budget, max_slots=slots, chunk=chunk, policy=policy,
                           time_scale=time_scale, pool_factory=factory, clock=clock.now, sleep=clock.sleep)
    return done, makespan, FakePool.instances[-1]


def test_every_request_completes_at_its_own_step_count():
    clock = Clock()
    reqs = make_requests([(0.0, 8, 8, 100, "a"), (0.001, 8, 8, 35, "b"), (0.002, 16, 8, 250, "c")])
    done, makespan, pool = run(reqs, clock)
    assert sorted(d.tag for d in done) == ["a", "b", "c"]
    assert pool.closed and pool.used == 0 and not pool.slots
    for d in done:
        assert d.admitted >= d.arrival and d.finished >= d.admitted
        # a solve needs its own steps at step_time each, rounded up to the
        # launch chunk, plus at most the chunks in flight when it joined
        assert d.latency >= d.steps * 1e-4 - 1e-9
        assert d.latency <= (d.steps + 3 * 10) * 1e-4 + 0.01
    s = summarize(done, makespan)
    assert s["requests"] == 3 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_fifo_admits_in_arrival_order_under_a_slot_limit():
    clock = Clock()
    reqs = make_requests([(0.0, 8, 8, 50, "a"), (0.0, 8, 8, 10, "b"), (0.0, 8, 8, 30, "c"), (0.0, 8, 8, 20, "d")])
    done, _, pool = run(reqs, clock, slots=1)
    order = [d.tag for d in sorted(done, key=lambda d: d.admitted)]
    assert order == ["a", "b", "c", "d"]


def test_sjf_admits_the_least_work_first():
    clock = Clock()
    reqs = make_requests([(0.0, 8, 8, 50, "a"), (0.0, 8, 8, 10, "b"), (0.0, 8, 8, 30, "c"), (0.0, 16, 8, 20, "d")])
    done, _, pool = run(reqs, clock, slots=1, policy="sjf")
    order = [d.tag for d in sorted(done, key=lambda d: d.admitted)]
    # work = nodes x steps: b 640, a 3200, c 1920, d 2560
    assert order == ["b", "c", "d", "a"]
    lat_sjf = np.mean([d.latency for d in done])
    clock = Clock()
    done_f, _, _ = run(make_requests([(0.0, 8, 8, 50, "a"), (0.0, 8, 8, 10, "b"), (0.0, 8, 8, 30, "c"),
                                      (0.0, 16, 8, 20, "d")]), clock, slots=1)
    assert lat_sjf < np.mean([d.latency for d in done_f])


def test_budget_holds_requests_back_until_memory_frees():
    clock = Clock()
    # 64 nodes each; a budget of 130 bytes holds two at a time
    reqs = make_requests([(0.0, 8, 8, 40, k) for k in "abcde"])
    done, _, pool = run(reqs, clock, budget=130)
    assert len(done) == 5 and pool.used == 0
    adm = sorted(d.admitted for d in done)
    assert adm[2] > adm[1]  # the third waited for a release


def test_time_scale_stretches_arrivals():
    clock = Clock()
    reqs = make_requests([(0.0, 8, 8, 10, "a"), (0.01, 8, 8, 10, "b")])
    done, _, _ = run(reqs, clock, time_scale=5.0)
    b = [d for d in done if d.tag == "b"][0]
    assert b.arrival == pytest.approx(0.05) and b.admitted >= 0.05


def test_a_request_larger_than_the_pool_is_refused():
    clock = Clock()
    reqs = make_requests([(0.0, 8, 8, 10, "small"), (0.0, 64, 64, 10, "huge")])
    with pytest.raises(ValueError, match="does not fit an empty pool"):
        run(reqs, clock, budget=1000)
    assert FakePool.instances[-1].closed


def test_a_solve_flagged_broken_is_retired_failed_and_the_others_finish():
    """A request whose slot the pool's diagnostics flag (a non-finite density)
    is retired as soon as the pool reports it, marked failed, and counted out
    of the throughput; the other requests complete at their own step counts."""
    clock = Clock()
    reqs = make_requests([(0.0, 8, 8, 400, "a"), (0.0, 8, 8, 400, "bad"), (0.0, 8, 8, 400, "c")])
    reqs[1].params = {"fail_at": 50}
    done, makespan, _ = run(reqs, clock)
    by = {d.tag: d for d in done}
    assert by["bad"].failed and not by["a"].failed and not by["c"].failed
    assert by["bad"].finished < by["a"].finished
    s = summarize(done, makespan)
    assert s["requests"] == 3 and s["failed"] == 1
    assert s["fluid_mlups"] == pytest.approx(2 * 64 * 400 / makespan / 1e6)
