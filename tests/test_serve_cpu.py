"""Host logic of the continuous-batching loop, driven by a fake executor on the CPU:
admission by footprint and slots, strict FIFO, iteration-level joining, failure
isolation, and the arena allocator."""
import numpy as np

from paper_2604_09643_amd.serve import POSE, Arena, Request, Scheduler


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Footprint = M*K bytes; step advances the clock by 1 ms per active request."""

    def __init__(self, clock, fail_on_step=None):
        self.clock = clock
        self.slots = {}
        self.steps = 0
        self.fail_on_step = fail_on_step
        self.log = []

    def footprint(self, req):
        return req.M * req.K

    def work(self, req):
        return float(req.M)

    def admit(self, req, slot):
        assert slot not in self.slots
        self.slots[slot] = {"req": req, "n": 0}
        self.log.append(("admit", req.rid, slot))
        return True

    def step(self, slots):
        self.steps += 1
        self.log.append(("step", tuple(self.slots[s]["req"].rid for s in slots)))
        if self.fail_on_step is not None and self.steps == self.fail_on_step:
            raise RuntimeError("injected launch failure")
        for s in slots:
            self.slots[s]["n"] += 1
        self.clock.t += 1e-3 * len(slots)

    def collect(self, slot, req):
        return np.full(6, float(self.slots[slot]["n"])), [0.0] * self.slots[slot]["n"], None

    def release(self, slot):
        self.slots.pop(slot)


def req(rid, M=64, K=512, steps=3, arrival=0.0, kind=POSE):
    return Request(rid, kind, (0, 0, 0, 8, 8, 8), np.zeros((M, 3)), np.zeros(6), np.zeros((M, K), np.float32),
                   steps, arrival)


def test_runs_every_request_with_its_step_count():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, slots=4, mem_cap=1 << 40, clock=clk)
    res = sch.run([req(i, steps=1 + i % 3, arrival=0.0) for i in range(10)], realtime=False)
    assert sorted(r.rid for r in res) == list(range(10))
    for r in res:
        assert r.pose6[0] == 1 + r.rid % 3          # exactly `steps` steps were run for it
    assert max(sch.batch_sizes) == 4                 # never more than the slot count


def test_iteration_level_joining():
    """A request arriving while another is mid-way joins the next tick, not after it ends."""
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, slots=4, mem_cap=1 << 40, clock=clk)
    sch.submit(req(0, steps=10, arrival=0.0))
    sch.submit(req(1, steps=2, arrival=0.0025))
    for _ in range(12):
        sch.tick()
    steps = [e[1] for e in ex.log if e[0] == "step"]
    first_joint = next(i for i, s in enumerate(steps) if 1 in s)
    assert 0 in steps[first_joint]                   # overlaps with request 0, which is mid-way
    assert first_joint <= 4
    done = {r.rid: r for r in sch.results}
    assert done[1].finished < done[0].finished       # the short request leaves first


def test_admission_by_footprint_with_lowered_cap():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    cap = 3 * 64 * 512                               # room for three requests of this size
    sch = Scheduler(ex, slots=16, mem_cap=cap, clock=clk)
    for i in range(6):
        sch.submit(req(i, steps=5))
    sch.tick()
    assert len(sch.active) == 3 and sch.mem_used == cap
    while sch.waiting or sch.active:
        sch.tick()
        assert sch.mem_used <= cap
    assert sorted(r.rid for r in sch.results) == list(range(6))


def test_oversized_request_is_rejected():
    clk = FakeClock()
    sch = Scheduler(FakeExecutor(clk), slots=2, mem_cap=1000, clock=clk)
    assert not sch.submit(req(0))
    assert sch.failed and sch.failed[0][0] == 0


def test_strict_fifo_no_overtaking():
    """A large request at the head blocks smaller later ones until it fits."""
    clk = FakeClock()
    ex = FakeExecutor(clk)
    cap = 2 * 64 * 512
    sch = Scheduler(ex, slots=8, mem_cap=cap, clock=clk)
    sch.submit(req(0, M=64, steps=4))
    sch.submit(req(1, M=128, steps=1))               # needs the whole cap
    sch.submit(req(2, M=16, steps=1))                # would fit now, but must wait behind 1
    sch.tick()
    admitted = [e[1] for e in ex.log if e[0] == "admit"]
    assert admitted == [0]
    while sch.waiting or sch.active:
        sch.tick()
    admitted = [e[1] for e in ex.log if e[0] == "admit"]
    assert admitted == [0, 1, 2]


def test_injected_failure_fails_only_that_batch():
    clk = FakeClock()
    ex = FakeExecutor(clk, fail_on_step=2)
    sch = Scheduler(ex, slots=2, mem_cap=1 << 40, clock=clk)
    res = sch.run([req(i, steps=2, arrival=0.01 * i) for i in range(5)], realtime=False)
    failed = {f[0] for f in sch.failed}
    ok = {r.rid for r in res}
    assert failed and not (failed & ok)
    assert failed | ok == set(range(5))
    assert max(ok) == 4                               # the loop kept serving after the failure
    assert not ex.slots                               # every slot was released


def test_arena_first_fit_and_merge():
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    a.release(x, 1000)
    assert a.alloc(2000) == 0                        # the two freed blocks merged
    a.release(0, 2000)
    a.release(z, 1000)
    assert a.free == [(0, 4096)] and a.used == 0


def test_work_budget_runs_large_requests_alone():
    """With a work budget, a request is admitted into a non-empty batch only while the batch's
    step work stays within the budget: a large request runs alone, small ones share ticks, and
    admission stays FIFO."""
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, slots=8, mem_cap=1 << 40, clock=clk, work_budget=100.0)
    reqs = [req(0, M=64, steps=3), req(1, M=128, steps=2), req(2, M=16, steps=2), req(3, M=16, steps=2),
            req(4, M=64, steps=1)]
    res = sch.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(5))
    steps = [e[1] for e in ex.log if e[0] == "step"]
    assert all(sum(reqs[r].M for r in b) <= 100 or len(b) == 1 for b in steps)
    assert any(b == (1,) for b in steps)               # 128 > budget: alone once admitted
    assert any(len(b) >= 2 for b in steps)              # small requests share ticks
    admitted = [e[1] for e in ex.log if e[0] == "admit"]
    assert admitted == [0, 1, 2, 3, 4]                  # FIFO
    assert sch.active_work == 0.0


def test_queue_lifts_the_work_budget():
    """With queue_lifts_budget, the budget applies while few requests wait and is lifted once that
    many have arrived and wait, so a backlog is served in shared ticks."""
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, slots=8, mem_cap=1 << 40, clock=clk, work_budget=100.0, queue_lifts_budget=3)
    for i in range(5):
        sch.submit(req(i, M=80, steps=2))
    sch.tick()                                          # 5 waiting: budget lifted, all join
    assert len(sch.active) == 5
    clk2 = FakeClock()
    ex2 = FakeExecutor(clk2)
    sch2 = Scheduler(ex2, slots=8, mem_cap=1 << 40, clock=clk2, work_budget=100.0, queue_lifts_budget=3)
    for i in range(2):
        sch2.submit(req(i, M=80, steps=2))
    sch2.tick()                                         # 2 waiting: the budget holds, one runs
    assert len(sch2.active) == 1


def test_queue_timeout_fails_waiting_requests():
    """With queue_timeout, an arrived request that is not admitted within that time fails with a
    queue-timeout reason and leaves the queue; admitted requests run on; without pressure nothing
    times out."""
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, slots=1, mem_cap=1 << 40, clock=clk, queue_timeout=0.0035)
    res = sch.run([req(0, steps=10), req(1, steps=1), req(2, steps=1, arrival=0.0005)], realtime=False)
    assert [r.rid for r in res] == [0]
    reasons = dict(sch.failed)
    assert set(reasons) == {1, 2} and all("queue timeout" in v for v in reasons.values())
    assert not sch.waiting and not sch.active and not ex.slots
    clk2 = FakeClock()
    sch2 = Scheduler(FakeExecutor(clk2), slots=1, mem_cap=1 << 40, clock=clk2, queue_timeout=0.05)
    res2 = sch2.run([req(0, steps=10), req(1, steps=1), req(2, steps=1)], realtime=False)
    assert sorted(r.rid for r in res2) == [0, 1, 2] and not sch2.failed
