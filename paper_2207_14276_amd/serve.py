"""Continuous batching of energy+force requests: bindings of the library's
native server (`nnp_server_*`) and of its host-only scheduler
(`nnp_sched_*`), plus a driver that replays a timed request trace.

A request is one system plus a number of successive evaluations (an MD-like
client whose atoms take a small random step between evaluations).  The
server keeps every admitted request's coordinates and neighbour list on the
device, evaluates the next step of all requests in flight in one batched
call per iteration, and admits waiting requests as slots and the memory
budget allow; see include/nnp.h for the exact semantics.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np

from . import _native as nat


class Scheduler:
    """The server's admission and step bookkeeping on its own (host only)."""

    def __init__(self, slots: int, max_batch_atoms: int, max_active: int = 1 << 30):
        lib = nat.load()
        h = C.c_void_p()
        nat.check(lib.nnp_sched_create(int(slots), int(max_batch_atoms), int(max_active), C.byref(h)))
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nnp_sched_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, rid: int, n_atoms: int, n_steps: int, t_arrival: float = 0.0):
        nat.check(self._lib.nnp_sched_submit(self._h, int(rid), int(n_atoms), int(n_steps),
                                             float(t_arrival)))

    def admit(self, now: float, max_n: int = 4096):
        ids = (C.c_int64 * max_n)()
        slots = (C.c_int64 * max_n)()
        n = C.c_int()
        nat.check(self._lib.nnp_sched_admit(self._h, float(now), ids, slots, max_n, C.byref(n)))
        return [(ids[k], slots[k]) for k in range(n.value)]

    def launch(self):
        """One step of every request in flight: [(id, slot, n_atoms, step)]."""
        m = max(1, self.info()["active"])
        ids, slots = (C.c_int64 * m)(), (C.c_int64 * m)()
        na, st = (C.c_int32 * m)(), (C.c_int32 * m)()
        n = C.c_int()
        nat.check(self._lib.nnp_sched_launch(self._h, ids, slots, na, st, m, C.byref(n)))
        return [(ids[k], slots[k], na[k], st[k]) for k in range(n.value)]

    def complete(self, rid: int, now: float) -> bool:
        fin = C.c_int()
        nat.check(self._lib.nnp_sched_complete(self._h, int(rid), float(now), C.byref(fin)))
        return bool(fin.value)

    def fail(self, rid: int, now: float):
        """Stops an admitted, unfinished request (its evaluation failed)."""
        nat.check(self._lib.nnp_sched_fail(self._h, int(rid), float(now)))

    def job(self, rid: int) -> dict:
        t = (C.c_double * 3)()
        slot = C.c_int64()
        done = C.c_int32()
        nat.check(self._lib.nnp_sched_job(self._h, int(rid), t, C.byref(slot), C.byref(done)))
        return {"arrival": t[0], "admitted": t[1], "done": t[2], "slot": slot.value,
                "steps_done": done.value}

    def info(self) -> dict:
        v = (C.c_int64 * 6)()
        nat.check(self._lib.nnp_sched_info(self._h, v))
        return dict(zip(["queued", "active", "active_atoms", "free_slots", "iterations",
                         "atom_evals"], list(v)))


@dataclass
class Request:
    coords: np.ndarray        # [n, 3] float32, Angstrom
    species: np.ndarray       # [n] int32 slot indices
    box: np.ndarray           # [3] float32 (0,0,0 = non-periodic)
    n_steps: int
    sigma: float = 0.01       # random-walk step per coordinate, Angstrom
    seed: int = 0

    @property
    def n_atoms(self) -> int:
        return int(len(self.species))


@dataclass
class Result:
    rid: int
    energies: np.ndarray      # [n_steps] float64, kcal/mol
    coords: np.ndarray        # [n, 3] float32, last step's coordinates
    forces: np.ndarray        # [n, 3] float32, last step's forces
    arrival: float
    admitted: float
    done: float
    error: int = 0            # NNP_ECAPACITY: the request stopped alone (neighbour overflow)
    message: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServerStats:
    iterations: int
    atom_evals: int
    queued: int
    active: int
    max_batch_atoms: int
    max_batch_seen: int
    device_bytes: int
    list_builds: int
    graph_captures: int
    graph_replays: int
    host_launch_s: float


class Server:
    """The library's continuous-batching server on one model (which it then
    uses exclusively).  `hbm_budget` bytes of device memory (0 = 90% of what
    is free) bound the per-iteration batch; see nnp_server_create.
    `use_graphs`: replay each iteration's kernels from a HIP graph recorded
    once per capacity bucket (else launch them one by one)."""

    def __init__(self, model, slots: int, capacity: int = 256, skin: float = 1.0,
                 max_batch_atoms: int = 0, max_active: int = 4096, hbm_budget: int = 0,
                 use_graphs: bool = True):
        import torch
        self.torch = torch
        self.model = model
        self._lib = nat.load()
        opts = nat.nnp_server_opts(int(slots), int(capacity), float(skin), int(max_batch_atoms),
                                   int(max_active), int(hbm_budget), 1 if use_graphs else 0)
        h = C.c_void_p()
        with torch.cuda.device(model.device):
            nat.check(self._lib.nnp_server_create(model.handle, C.byref(opts), C.byref(h)))
        self._h = h
        self.n_atoms = {}
        self.n_steps = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            with self.torch.cuda.device(self.model.device):
                self._lib.nnp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        return float(self._lib.nnp_server_clock(self._h))

    def submit(self, req: Request, t_arrival: float = -1.0) -> int:
        x = np.ascontiguousarray(req.coords, dtype=np.float32).reshape(-1, 3)
        s = np.ascontiguousarray(req.species, dtype=np.int32)
        if len(x) != len(s):
            raise ValueError("coords and species differ in length")
        r = nat.nnp_request(len(s), x.ctypes.data_as(C.POINTER(C.c_float)),
                            s.ctypes.data_as(C.POINTER(C.c_int32)),
                            (C.c_float * 3)(*[float(v) for v in np.asarray(req.box).reshape(3)]),
                            int(req.n_steps), float(req.sigma), int(req.seed) & ((1 << 64) - 1))
        rid = C.c_int64()
        nat.check(self._lib.nnp_server_submit(self._h, C.byref(r), float(t_arrival), C.byref(rid)))
        self.n_atoms[rid.value] = len(s)
        self.n_steps[rid.value] = int(req.n_steps)
        return rid.value

    def step(self) -> int:
        """One iteration on torch's current stream; returns the number of
        requests queued or in flight plus iterations not yet filed."""
        torch = self.torch
        pend = C.c_int64()
        with torch.cuda.device(self.model.device):
            st = C.c_void_p(torch.cuda.current_stream(self.model.device).cuda_stream)
            nat.check(self._lib.nnp_server_step(self._h, st, C.byref(pend)))
        return int(pend.value)

    def drain(self):
        nat.check(self._lib.nnp_server_drain(self._h))

    def poll(self, max_n: int = 4096):
        ids = (C.c_int64 * max_n)()
        n = C.c_int()
        nat.check(self._lib.nnp_server_poll(self._h, ids, max_n, C.byref(n)))
        return [ids[k] for k in range(n.value)]

    def result(self, rid: int) -> Result:
        n, k = self.n_atoms.pop(rid), self.n_steps.pop(rid)
        e = np.empty(k, np.float64)
        x = np.empty((n, 3), np.float32)
        f = np.empty((n, 3), np.float32)
        t = np.empty(3, np.float64)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        rc = self._lib.nnp_server_result(self._h, int(rid), e.ctypes.data_as(dp), x.ctypes.data_as(fp),
                                         f.ctypes.data_as(fp), t.ctypes.data_as(dp))
        if rc == nat.NNP_ECAPACITY:
            # this request stopped alone; the server and the other requests go on
            return Result(rid, np.zeros(0), np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                          float(t[0]), float(t[1]), float(t[2]), rc, nat.last_error())
        nat.check(rc)
        return Result(rid, e, x, f, float(t[0]), float(t[1]), float(t[2]))

    def stats(self) -> ServerStats:
        c = nat.nnp_server_counters()
        nat.check(self._lib.nnp_server_stats(self._h, C.byref(c)))
        return ServerStats(*[getattr(c, f) for f, _ in nat.nnp_server_counters._fields_])


@dataclass
class Replay:
    results: dict = field(default_factory=dict)   # rid -> Result
    order: list = field(default_factory=list)     # rids in trace order
    wall: float = 0.0                             # first arrival -> last completion, s
    steps: int = 0                                # nnp_server_step calls

    def latencies(self, skip: int = 0) -> np.ndarray:
        return np.array([self.results[r].latency for r in self.order[skip:]])


def replay(server: Server, arrivals, max_steps: int | None = None) -> Replay:
    """Feeds `arrivals` ([(t, Request)] sorted by t, seconds from the start)
    to the server on its own clock: each request is submitted once its time
    has come (stamped with its scheduled arrival), and the server is stepped
    until everything submitted has finished."""
    out = Replay()
    pending = list(arrivals)
    k = 0
    t0 = server.clock()
    busy = 0
    while k < len(pending) or busy:
        now = server.clock() - t0
        while k < len(pending) and pending[k][0] <= now:
            t, req = pending[k]
            out.order.append(server.submit(req, t0 + t))
            k += 1
            busy = max(busy, 1)   # a submitted request is work for the next step
        if not busy:
            # nothing queued or in flight: idle until the next arrival
            time.sleep(max(0.0, pending[k][0] - (server.clock() - t0)))
            continue
        busy = server.step()
        out.steps += 1
        for rid in server.poll():
            out.results[rid] = server.result(rid)
        if max_steps is not None and out.steps >= max_steps:
            break
    server.drain()
    for rid in server.poll():
        out.results[rid] = server.result(rid)
    if out.results:
        out.wall = max(r.done for r in out.results.values()) - (t0 + pending[0][0])
    return out
