"""Scheduler logic of the continuous-batching server, on a fake clock and a
fake executor (pure host logic; no GPU)."""
import pytest

from paper_2311_14140_amd.serve import Executor, Request, Server
from synth import Params


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor(Executor):
    """Instances cost `sec_per_particle_step` of device time per step."""

    def __init__(self, clock, sec_per_particle_step=1e-9, bytes_per_particle=40):
        self.clock = clock
        self.c = sec_per_particle_step
        self.bpp = bytes_per_particle
        self.running = {}
        self.log = []
        self._next = 0

    def footprint(self, p):
        return p.n_cells * p.particles_per_cell * self.bpp

    def start(self, p):
        h = self._next
        self._next += 1
        self.running[h] = [p, 0]
        self.log.append(("start", h, self.clock.t, len(self.running)))
        return h

    def step(self, n):
        work = sum(v[0].n_cells * v[0].particles_per_cell for v in self.running.values())
        for v in self.running.values():
            v[1] += n
        self.clock.t += n * work * self.c

    def finish(self, h):
        p, steps = self.running.pop(h)
        self.log.append(("finish", h, self.clock.t, steps))
        return {"steps": steps, "seed": p.seed}


def P(cells, ppc, seed=0):
    return Params(kn=1.0, body_force=0.01, n_cells=cells, particles_per_cell=ppc, seed=seed)


def test_every_request_gets_exactly_its_steps():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = [Request(i, 0.001 * i, P(10 + i, 20, seed=i), steps=37 * (i + 1)) for i in range(12)]
    srv = Server(ex, budget_bytes=10**9, max_slots=5, quantum=50, clock=clk, sleep=clk.sleep)
    res, summ = srv.run(reqs)
    assert summ["served"] == 12 and summ["rejected"] == 0
    by = {r.rid: r for r in res}
    for q in reqs:
        assert by[q.rid].moments["steps"] == q.steps
        assert by[q.rid].moments["seed"] == q.params.seed
        assert by[q.rid].finished >= by[q.rid].admitted >= q.arrival
    # never more than max_slots together
    assert max(e[3] for e in ex.log if e[0] == "start") <= 5


def test_admission_by_footprint_budget():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    big = P(100, 100)     # 4e5 bytes
    reqs = [Request(i, 0.0, big, steps=100) for i in range(6)]
    srv = Server(ex, budget_bytes=1_000_000, max_slots=64, quantum=100, clock=clk, sleep=clk.sleep)
    res, summ = srv.run(reqs)
    # two fit at a time: the running set never exceeds the budget
    assert max(e[3] for e in ex.log if e[0] == "start") == 2
    assert summ["peak_bytes"] <= 1_000_000
    assert summ["served"] == 6


def test_too_large_request_is_rejected_not_blocking():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = [Request(0, 0.0, P(1000, 1000), steps=10), Request(1, 0.0, P(10, 10), steps=10)]
    srv = Server(ex, budget_bytes=100_000, clock=clk, sleep=clk.sleep)
    res, summ = srv.run(reqs)
    assert summ["rejected"] == 1 and summ["served"] == 1
    assert [r.rid for r in res if r.rejected] == [0]


def test_fifo_admission_and_idle_wait():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = [Request(0, 0.5, P(10, 10), steps=10), Request(1, 0.2, P(10, 10), steps=10),
            Request(2, 5.0, P(10, 10), steps=10)]
    srv = Server(ex, budget_bytes=10**9, max_slots=1, quantum=10, clock=clk, sleep=clk.sleep)
    res, summ = srv.run(reqs)
    starts = [e[1] for e in ex.log if e[0] == "start"]
    assert starts == [0, 1, 2]         # handles in admission order: rid 1, 0, 2
    by = {r.rid: r for r in res}
    assert by[1].admitted == pytest.approx(0.2) and by[2].admitted == pytest.approx(5.0)
    assert by[0].admitted >= by[1].finished


def test_newcomers_join_running_group_between_quanta():
    clk = FakeClock()
    ex = FakeExecutor(clk, sec_per_particle_step=1e-6)
    reqs = [Request(0, 0.0, P(100, 10), steps=1000), Request(1, 0.05, P(100, 10), steps=100)]
    srv = Server(ex, budget_bytes=10**9, quantum=10, clock=clk, sleep=clk.sleep)
    res, summ = srv.run(reqs)
    by = {r.rid: r for r in res}
    # the short request is admitted while the long one runs and finishes first
    assert by[1].admitted < by[0].finished
    assert by[1].finished < by[0].finished
    assert summ["p99_s"] >= summ["p50_s"] > 0
    assert 0 < summ["utilisation"] <= 1.0


def test_invalid_server_arguments():
    clk = FakeClock()
    with pytest.raises(ValueError):
        Server(FakeExecutor(clk), budget_bytes=0)
    with pytest.raises(ValueError):
        Server(FakeExecutor(clk), budget_bytes=10, quantum=0)
