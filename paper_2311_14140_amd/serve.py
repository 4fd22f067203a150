"""Continuous-batching service for DSMC solves.

Requests (solver parameters plus a number of steps) arrive over time.  The
server admits them in arrival order as soon as two things are free: a slot
(at most ``max_slots`` instances run together) and device memory (the
instance's footprint fits in what is left of ``budget_bytes``).  Admitted
instances keep their particle state resident on the device and join the
running group; the group advances in quanta of steps, every member by the
same number, so the work of all running requests shares each launch.  A
request whose steps are done has its sampled moments copied to the host, is
removed and destroyed, and its memory and slot go to the next request.
Requests that arrive while others are on the device therefore overlap with
them.

Each instance's arithmetic and ordering do not depend on the group it runs
in, so a request's result is the same (bit for bit) alone and in the mix.

The scheduling logic is independent of the device: ``Server`` drives any
``Executor``; ``GpuExecutor`` runs the instances on the GPU through the C ABI
as one group, ``PlainGpuExecutor`` steps each instance on its own.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

from . import stats


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    params: object          # any object with the fields of synth.Params
    steps: int              # steps to run (transient + sampling)


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    moments: dict = field(repr=False, default=None)
    particle_steps: int = 0
    rejected: bool = False

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Executor:
    """What the server needs from a device."""

    def footprint(self, params) -> int:
        raise NotImplementedError

    def start(self, params):
        """Create an instance and add it to the running set; returns a handle."""
        raise NotImplementedError

    def step(self, n: int) -> None:
        """Advance every running instance by n steps and wait for them."""
        raise NotImplementedError

    def finish(self, handle) -> dict:
        """Sampled moments of a running instance, which is then released."""
        raise NotImplementedError


class GpuExecutor(Executor):
    """Instances on the current GPU, stepped as one group per quantum.
    Device memory comes from torch tensors (one arena per instance)."""

    def __init__(self, stream=None, tune: bool = False):
        from . import dsmc
        self._d = dsmc
        self._group = dsmc.Group(stream)
        self._stream = stream
        self._tune = tune
        self._tuned = False

    def footprint(self, params) -> int:
        return self._d.footprint_bytes(params)

    def start(self, params):
        s = self._d.Solver(params, stream=self._stream, arena="torch")
        self._group.add(s)
        self._tuned = False
        return s

    def step(self, n: int) -> None:
        if self._tune and not self._tuned and len(self._group.members) > 1:
            self._group.autotune()
            self._tuned = True
        self._group.step(n)
        self._group.sync()

    def finish(self, handle) -> dict:
        self._group.remove(handle)
        out = handle.sample()
        handle.close()
        return out

    def close(self):
        self._group.close()


class PlainGpuExecutor(Executor):
    """Every instance stepped on its own (no group): with ``max_slots=1`` this
    is the plain one-solve-at-a-time service the batched one is compared with."""

    def __init__(self, stream=None):
        from . import dsmc
        self._d = dsmc
        self._stream = stream
        self._running = []

    def footprint(self, params) -> int:
        return self._d.footprint_bytes(params)

    def start(self, params):
        s = self._d.Solver(params, stream=self._stream, arena="torch")
        self._running.append(s)
        return s

    def step(self, n: int) -> None:
        for s in self._running:
            s.step(n)
        for s in self._running:
            s.sync()

    def finish(self, handle) -> dict:
        self._running.remove(handle)
        out = handle.sample()
        handle.close()
        return out


class Server:
    def __init__(self, executor: Executor, budget_bytes: int, max_slots: int = 256,
                 quantum: int = 100, clock=time.perf_counter, sleep=time.sleep):
        if budget_bytes <= 0 or max_slots <= 0 or quantum <= 0:
            raise ValueError("budget, slots and quantum must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.quantum = int(quantum)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests):
        """Serve the requests (sorted by arrival) to completion.  Returns
        (results in completion order, summary dict)."""
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        running = {}   # rid -> [handle, request, steps_done, admitted_at, footprint]
        results = []
        used = 0
        peak_used = 0
        busy = 0.0
        t0 = self.clock()

        def now():
            return self.clock() - t0

        while pending or running:
            t = now()
            # admit, in arrival order, while a slot and memory are free
            while pending and pending[0].arrival <= t and len(running) < self.max_slots:
                r = pending[0]
                fp = self.ex.footprint(r.params)
                if fp > self.budget:
                    pending.popleft()
                    results.append(Result(r.rid, r.arrival, t, t, None, 0, rejected=True))
                    continue
                if used + fp > self.budget:
                    break
                pending.popleft()
                h = self.ex.start(r.params)
                running[r.rid] = [h, r, 0, now(), fp]
                used += fp
                peak_used = max(peak_used, used)
            if not running:
                if pending:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        self.sleep(wait)
                continue
            q = min(self.quantum, min(v[1].steps - v[2] for v in running.values()))
            a = self.clock()
            self.ex.step(q)
            busy += self.clock() - a
            done = []
            for rid, v in running.items():
                v[2] += q
                if v[2] >= v[1].steps:
                    done.append(rid)
            for rid in done:
                h, r, steps, adm, fp = running.pop(rid)
                mom = self.ex.finish(h)
                results.append(Result(rid, r.arrival, adm, now(), mom,
                                      particle_steps=steps * self._particles(r.params)))
                used -= fp
        makespan = now()
        served = [r for r in results if not r.rejected]
        lat = [r.latency for r in served]
        ps = sum(r.particle_steps for r in served)
        summary = {
            "requests": len(results), "served": len(served),
            "rejected": sum(r.rejected for r in results),
            "p50_s": stats.percentile(lat, 50), "p99_s": stats.percentile(lat, 99),
            "mean_s": float(sum(lat) / len(lat)) if lat else float("nan"),
            "makespan_s": makespan, "particle_steps": ps,
            "throughput": ps / makespan if makespan > 0 else float("nan"),
            "utilisation": busy / makespan if makespan > 0 else float("nan"),
            "peak_bytes": peak_used,
        }
        return results, summary

    @staticmethod
    def _particles(params) -> int:
        return int(params.n_cells) * int(params.particles_per_cell)
