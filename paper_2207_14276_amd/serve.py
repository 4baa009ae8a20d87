"""Continuous batching of energy+force requests on one GPU.

A request is one system plus a number of successive steps (an MD client that
moves the atoms a little between steps and needs energy and forces each
time).  The server keeps every in-flight request's coordinates, species and
neighbour list on the device; each iteration it evaluates the next step of
every in-flight request in one batched library call, then advances each
request (its client moves the atoms on the device).  Requests that arrive
meanwhile wait in a queue and are admitted as soon as neighbour-list slots
and the atom budget of one batch allow, so new work joins the running batch
at the next iteration.

Scheduling (queue, admission, slots, latency bookkeeping) is host logic in
`Scheduler`, independent of the GPU so it can be tested on its own;
`GpuExecutor` owns the device state and issues the library calls.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    """One request: a system and the number of steps its client asks for."""
    rid: int
    n_atoms: int
    n_steps: int
    arrival: float
    payload: object = None       # executor-specific (coordinates, species, box, seed)
    slot: int = -1               # first neighbour-list slot
    admitted: float = -1.0
    steps_done: int = 0
    done_time: float = -1.0
    fresh: bool = True           # next evaluation must build its neighbour list


class SlotAllocator:
    """First-fit allocator of contiguous slot ranges in [0, total)."""

    def __init__(self, total: int):
        self.total = int(total)
        self.free = [(0, self.total)]  # sorted (start, length)

    def alloc(self, n: int):
        for k, (s, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (s + n, ln - n)
                return s
        return None

    def release(self, start: int, n: int):
        self.free.append((start, n))
        self.free.sort()
        merged = []
        for s, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((s, ln))
        self.free = merged

    @property
    def free_slots(self) -> int:
        return sum(ln for _, ln in self.free)


class Scheduler:
    """Queue, admission and step accounting.

    Admission is first-come first-served: the head of the queue is admitted
    when a contiguous slot range of its size is free and the batch stays within
    `max_batch_atoms`; otherwise it (and everything behind it) waits.  A job
    larger than either limit can never run and is rejected at submission.
    """

    def __init__(self, slots: int, max_batch_atoms: int, clock=time.perf_counter):
        self.alloc = SlotAllocator(slots)
        self.max_batch_atoms = int(max_batch_atoms)
        self.clock = clock
        self.queue: deque[Job] = deque()
        self.active: list[Job] = []
        self.finished: list[Job] = []
        self.atom_evals = 0
        self.iterations = 0

    def submit(self, job: Job):
        if job.n_atoms > self.alloc.total or job.n_atoms > self.max_batch_atoms:
            raise ValueError(f"request of {job.n_atoms} atoms exceeds the server's capacity")
        self.queue.append(job)

    @property
    def active_atoms(self) -> int:
        return sum(j.n_atoms for j in self.active)

    def admit(self) -> list[Job]:
        out = []
        while self.queue:
            j = self.queue[0]
            if self.active_atoms + j.n_atoms > self.max_batch_atoms:
                break
            s = self.alloc.alloc(j.n_atoms)
            if s is None:
                break
            self.queue.popleft()
            j.slot = s
            j.admitted = self.clock()
            j.fresh = True
            self.active.append(j)
            out.append(j)
        return out

    def batch(self) -> list[Job]:
        """Jobs evaluated in the next iteration: every in-flight job."""
        return list(self.active)

    def complete(self, batch: list[Job], t_done: float) -> list[Job]:
        """Marks one step of every job in `batch` done; returns jobs that finished."""
        self.iterations += 1
        fin = []
        for j in batch:
            self.atom_evals += j.n_atoms
            j.steps_done += 1
            j.fresh = False
            if j.steps_done >= j.n_steps:
                j.done_time = t_done
                fin.append(j)
        for j in fin:
            self.active.remove(j)
            self.alloc.release(j.slot, j.n_atoms)
            self.finished.append(j)
        return fin

    def latencies(self, skip: int = 0) -> np.ndarray:
        done = sorted(self.finished, key=lambda j: j.arrival)[skip:]
        return np.array([j.done_time - j.arrival for j in done])


@dataclass
class SystemPayload:
    coords: np.ndarray
    species: np.ndarray
    box: np.ndarray
    seed: int
    sigma: float = 0.01
    record: bool = False           # keep every step's inputs and outputs (tests)
    trace: list = field(default_factory=list)


class GpuExecutor:
    """Device state of the in-flight jobs and the batched library calls."""

    def __init__(self, model, slots: int, capacity: int = 256, skin: float = 1.0):
        import torch
        from .model import NeighborPool
        self.torch = torch
        self.model = model
        self.pool = NeighborPool(model, slots, capacity, skin)
        self.dev = model.device
        self.state = {}  # rid -> (coords tensor, species tensor, box, generator)

    def admit(self, job: Job):
        t = self.torch
        p: SystemPayload = job.payload
        c = t.as_tensor(p.coords, dtype=t.float32, device=self.dev).contiguous()
        s = t.as_tensor(p.species, dtype=t.int32, device=self.dev).contiguous()
        g = t.Generator(device=self.dev)
        g.manual_seed(int(p.seed))
        self.state[job.rid] = (c, s, np.asarray(p.box, np.float32), g)

    def evaluate(self, batch: list[Job]):
        """Enqueues one batched evaluation; returns the result (device tensors)."""
        t = self.torch
        coords = t.cat([self.state[j.rid][0] for j in batch])
        species = t.cat([self.state[j.rid][1] for j in batch])
        boxes = np.stack([self.state[j.rid][2] for j in batch])
        offs = np.zeros(len(batch) + 1, np.int64)
        offs[1:] = np.cumsum([j.n_atoms for j in batch])
        slots = np.array([j.slot for j in batch], np.int64)
        rebuild = np.array([1 if j.fresh else 0 for j in batch], np.int32)
        res = self.pool.energy_forces(coords, species, boxes, offs, slots, rebuild, forces=True)
        for k, j in enumerate(batch):
            p: SystemPayload = j.payload
            if p.record:
                a, e = int(offs[k]), int(offs[k + 1])
                p.trace.append((coords[a:e].clone(), res.energy[k:k + 1].clone(),
                                res.forces[a:e].clone()))
        return res

    def advance(self, batch: list[Job], finished: list[Job]):
        """The clients take their step: each continuing system moves by
        N(0, sigma) per coordinate (a random walk, on the device)."""
        t = self.torch
        done = {j.rid for j in finished}
        for j in batch:
            c, s, b, g = self.state[j.rid]
            if j.rid in done:
                del self.state[j.rid]
                continue
            c.add_(t.randn(c.shape, generator=g, device=self.dev) * j.payload.sigma)

    def builds(self) -> int:
        return self.pool.builds()

    def check(self):
        """Waits for the device and raises on a device flag (neighbour
        capacity overflow, bad species) of the calls so far."""
        self.model.status()


def serve(executor, sched: Scheduler, arrivals, clock=time.perf_counter, sync=None,
          max_iterations: int | None = None):
    """Replays `arrivals` (list of (t_arrival, Job), sorted, times relative to
    the start) through the scheduler; returns when every job has finished."""
    pending = deque(arrivals)
    t0 = clock()
    it = 0
    while pending or sched.queue or sched.active:
        now = clock() - t0
        while pending and pending[0][0] <= now:
            ta, job = pending.popleft()
            job.arrival = t0 + ta
            sched.submit(job)
        for j in sched.admit():
            executor.admit(j)
        if not sched.active:
            if pending:
                time.sleep(max(0.0, pending[0][0] - (clock() - t0)))
            continue
        batch = sched.batch()
        executor.evaluate(batch)
        if sync is not None:
            sync()
            if hasattr(executor, "check"):
                executor.check()
        fin = sched.complete(batch, clock())
        executor.advance(batch, fin)
        it += 1
        if max_iterations is not None and it >= max_iterations:
            break
    return clock() - t0
