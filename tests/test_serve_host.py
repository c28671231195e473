"""Host logic of the continuous-batching loop (admission by footprint, first
come first served, joining at step boundaries, capacity retry with rollback),
driven by a stand-in batch and a simulated clock.  No GPU is used."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2607_26901_amd import ccfr
from paper_2607_26901_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBatch:
    """Records which requests are resident at every step; one step takes 1 s."""

    def __init__(self, clock, max_slots, overflow_at=()):
        self.clock = clock
        self.max_slots = max_slots
        self.slots = {}
        self.log = []
        self.overflow_at = set(overflow_at)
        self.rollbacks = 0
        self.pending_overflow = False
        self.n_steps = 0

    def add_scene(self, scene, sp):
        free = [k for k in range(self.max_slots) if k not in self.slots]
        if not free:
            raise ccfr.CcfrError(-2, "add")
        self.slots[free[0]] = scene
        return free[0]

    def step(self):
        self.clock.t += 1.0
        self.n_steps += 1
        self.pending_overflow = self.n_steps in self.overflow_at
        self.log.append(sorted(s.name for s in self.slots.values()))

    def rollback(self):
        self.rollbacks += 1
        self.log.pop()

    def read(self, slot):
        n = self.slots[slot].n_verts
        return np.zeros((n, 3), np.float32), np.zeros((n, 3), np.float32)

    def remove(self, slot):
        del self.slots[slot]


class FakeCtx:
    def __init__(self, batch):
        self.batch = batch
        self.reserved = []

    def sync_status(self, reset=False):
        if self.batch.pending_overflow:
            self.batch.pending_overflow = False
            return -2, {"need": [10, 20, 30, 40, 50, 0]}
        return 0, {"need": [0] * 6}

    def grow(self, info):
        self.reserved.append({"vf": int(info["need"][0] * 1.5) + 1024})


def job(i, arrival, n_verts, steps):
    sc = SimpleNamespace(name=f"r{i}", n_verts=n_verts, n_dynamic=n_verts, tris=np.zeros((0, 3)),
                         edges=np.zeros((0, 2)), step=SimpleNamespace(iters=2), params=None)
    return serve.Job(i, arrival, sc, steps)


def make_server(clock, budget, max_slots=8, overflow_at=()):
    b = FakeBatch(clock, max_slots, overflow_at)
    ctx = FakeCtx(b)
    srv = serve.Server(ctx, budget, batch=b, timer=serve._HostTimer(), footprint_fn=lambda sc: sc.n_verts)
    return srv, b, ctx


@pytest.fixture(autouse=True)
def _plain_step_params(monkeypatch):
    monkeypatch.setattr(ccfr, "make_step_params", lambda step, params: None)


def test_budget_and_fifo():
    clock = Clock()
    srv, b, _ = make_server(clock, budget=100)
    jobs = [job(0, 0.0, 60, 3), job(1, 0.0, 50, 2), job(2, 0.0, 30, 2)]
    st = srv.run(jobs, clock=clock, sleep=clock.sleep)
    # r1 does not fit beside r0 (110 > 100) and r2 may not overtake it
    assert b.log[:3] == [["r0"], ["r0"], ["r0"]]
    assert b.log[3:] == [["r1", "r2"], ["r1", "r2"]]
    assert set(st.results) == {0, 1, 2}
    assert st.updates == 2 * (60 * 3 + 50 * 2 + 30 * 2)


def test_late_arrival_joins_running_batch():
    clock = Clock()
    srv, b, _ = make_server(clock, budget=1000)
    jobs = [job(0, 0.0, 10, 4), job(1, 1.5, 10, 2)]
    st = srv.run(jobs, clock=clock, sleep=clock.sleep)
    assert b.log == [["r0"], ["r0"], ["r0", "r1"], ["r0", "r1"]]
    assert st.results[1].finished == 4.0 and st.results[0].finished == 4.0
    assert st.max_resident == 2


def test_idle_until_first_arrival_and_slot_limit():
    clock = Clock()
    srv, b, _ = make_server(clock, budget=10 ** 9, max_slots=2)
    jobs = [job(i, 5.0, 10, 1) for i in range(3)]
    st = srv.run(jobs, clock=clock, sleep=clock.sleep)
    assert b.log == [["r0", "r1"], ["r2"]]
    assert min(r.admitted for r in st.results.values()) == 5.0


def test_capacity_overflow_rolls_back_and_repeats():
    clock = Clock()
    srv, b, ctx = make_server(clock, budget=1000, overflow_at=(2,))
    st = srv.run([job(0, 0.0, 10, 3)], clock=clock, sleep=clock.sleep)
    assert b.rollbacks == 1 and st.retries == 1
    assert len(ctx.reserved) == 1 and ctx.reserved[0]["vf"] >= 15
    assert b.log == [["r0"]] * 3                  # exactly the requested steps survive
    assert st.results[0].steps == 3


def test_oversize_request_runs_alone():
    clock = Clock()
    srv, b, _ = make_server(clock, budget=50)
    st = srv.run([job(0, 0.0, 80, 1), job(1, 0.0, 10, 1)], clock=clock, sleep=clock.sleep)
    assert b.log == [["r0"], ["r1"]]
    assert len(st.results) == 2
