"""Host logic of the serving layer through the C ABI, without a GPU: the
native scheduler's first-fit slot ranges, first-come first-served admission
under the slot, batch-atom and in-flight limits, continuous joining of new
requests, step accounting and latencies (driven with explicit times)."""
import numpy as np
import pytest

from paper_2207_14276_amd import NNPError
from paper_2207_14276_amd.serve import Scheduler


def run_to_completion(s, arrivals, dt=1.0):
    """Replays [(t_arrival, rid, n_atoms, n_steps)] with one iteration per
    `dt` of time; returns the batches (lists of ids) launched."""
    t, k, batches = 0.0, 0, []
    arrivals = sorted(arrivals)
    while True:
        while k < len(arrivals) and arrivals[k][0] <= t:
            ta, rid, n, st = arrivals[k]
            s.submit(rid, n, st, ta)
            k += 1
        s.admit(t)
        items = s.launch()
        if not items:
            if k == len(arrivals) and s.info()["queued"] == 0:
                return batches
            t = arrivals[k][0] if k < len(arrivals) else t + dt
            continue
        batches.append([it[0] for it in items])
        t += dt
        for it in items:
            s.complete(it[0], t)


def test_first_fit_slots_and_merge():
    s = Scheduler(slots=100, max_batch_atoms=1000)
    for rid, (n, steps) in enumerate([(30, 3), (30, 1), (30, 3)]):
        s.submit(rid, n, steps)
    assert s.admit(0.0) == [(0, 0), (1, 30), (2, 60)]
    s.launch()                      # request 1 launches its only step: slots 30..59 free
    assert s.info()["free_slots"] == 40
    s.submit(3, 35, 1)              # the 30-slot hole and the 10 at the end do not fit 35
    s.submit(4, 25, 1)              # first come first served: 4 waits behind 3
    assert s.admit(1.0) == []
    s.launch()
    s.launch()                      # requests 0 and 2 finish: everything merges back
    assert s.info()["free_slots"] == 100
    assert s.admit(2.0) == [(3, 0), (4, 35)]


def test_fcfs_admission_respects_slot_and_batch_budgets():
    s = Scheduler(slots=100, max_batch_atoms=80)
    for rid, n in enumerate([50, 40, 20, 10]):
        s.submit(rid, n, 2, 0.0)
    # 50 fits; 40 would exceed the 80-atom batch budget; 20 and 10 wait behind it
    assert [r for r, _ in s.admit(0.0)] == [0]
    s.launch()
    assert s.admit(1.0) == []
    s.launch()                      # request 0 launches its last step
    assert [r for r, _ in s.admit(2.0)] == [1, 2, 3]


def test_in_flight_limit():
    s = Scheduler(slots=1000, max_batch_atoms=1000, max_active=2)
    for rid in range(4):
        s.submit(rid, 10, 1)
    assert [r for r, _ in s.admit(0.0)] == [0, 1]
    s.launch()
    assert [r for r, _ in s.admit(1.0)] == [2, 3]


def test_requests_that_can_never_run_are_refused():
    s = Scheduler(slots=100, max_batch_atoms=50)
    with pytest.raises(NNPError):
        s.submit(0, 60, 1)          # above the batch budget
    with pytest.raises(NNPError):
        s.submit(1, 10, 0)          # no steps
    s.submit(2, 10, 1)
    with pytest.raises(NNPError):
        s.submit(2, 10, 1)          # id in use
    s2 = Scheduler(slots=40, max_batch_atoms=1000)
    with pytest.raises(NNPError):
        s2.submit(0, 41, 1)         # above the pool


def test_continuous_batching_joins_new_requests_mid_flight():
    s = Scheduler(slots=1000, max_batch_atoms=1000)
    batches = run_to_completion(s, [(0.0, 0, 10, 5), (2.5, 1, 20, 2), (2.5, 2, 5, 1)])
    # request 0 runs alone for three iterations, then 1 and 2 join the batch
    assert batches == [[0], [0], [0], [0, 1, 2], [0, 1]]
    lat = {r: s.job(r)["done"] - s.job(r)["arrival"] for r in range(3)}
    assert lat[0] == pytest.approx(5.0)
    assert lat[1] == pytest.approx(2.5)
    assert lat[2] == pytest.approx(1.5)
    assert s.info()["atom_evals"] == 10 * 5 + 20 * 2 + 5 * 1
    assert s.info()["iterations"] == 5


def test_queue_waits_for_slots_then_drains():
    s = Scheduler(slots=30, max_batch_atoms=1000)
    batches = run_to_completion(s, [(0.0, k, 20, 3) for k in range(4)])
    # one 20-atom request fits the 30 slots at a time: strictly sequential
    assert all(len(b) == 1 for b in batches)
    lat = sorted(s.job(r)["done"] - s.job(r)["arrival"] for r in range(4))
    np.testing.assert_allclose(lat, [3, 6, 9, 12])


def test_complete_without_a_launched_step_is_an_error():
    s = Scheduler(slots=10, max_batch_atoms=10)
    s.submit(0, 5, 2)
    s.admit(0.0)
    with pytest.raises(NNPError):
        s.complete(0, 0.0)
    s.launch()
    assert s.complete(0, 1.0) is False
    s.launch()
    assert s.complete(0, 2.0) is True
    assert s.job(0)["steps_done"] == 2


def test_randomized_invariants():
    """Random arrivals and sizes: slot ranges of requests in flight never
    overlap, the batch budget holds every iteration, every request runs
    exactly its steps, and admission order is arrival order."""
    rng = np.random.default_rng(0)
    slots, budget = 500, 300
    s = Scheduler(slots=slots, max_batch_atoms=budget, max_active=16)
    n_req = 200
    sizes = rng.integers(1, 120, n_req)
    steps = rng.integers(1, 6, n_req)
    t, k, admitted_order, live = 0.0, 0, [], {}
    launched = {r: 0 for r in range(n_req)}
    while k < n_req or s.info()["queued"] or s.info()["active"]:
        for _ in range(int(rng.integers(0, 4))):
            if k < n_req:
                s.submit(k, int(sizes[k]), int(steps[k]), t)
                k += 1
        for rid, slot in s.admit(t):
            admitted_order.append(rid)
            live[rid] = (slot, int(sizes[rid]))
        ranges = sorted(live.values())
        for (a0, n0), (a1, _) in zip(ranges, ranges[1:]):
            assert a0 + n0 <= a1
        assert all(0 <= a and a + n <= slots for a, n in ranges)
        items = s.launch()
        assert sum(it[2] for it in items) <= budget
        t += 1.0
        for rid, slot, n, st in items:
            assert st == launched[rid]
            launched[rid] += 1
            if s.complete(rid, t):
                del live[rid]
    assert admitted_order == list(range(n_req))
    assert all(launched[r] == steps[r] for r in range(n_req))


class _FakeServer:
    """Stand-in for serve.Server on a virtual clock: every step advances the
    clock by `dt` and moves each request in flight on by one evaluation."""

    def __init__(self, dt):
        self.t, self.dt = 0.0, dt
        self.active, self.done, self.next_id = {}, [], 0
        self.batches, self.finished = [], {}

    def clock(self):
        return self.t

    def submit(self, req, t_arrival):
        rid = self.next_id
        self.next_id += 1
        self.active[rid] = [req, t_arrival]
        return rid

    def step(self):
        self.batches.append(sorted(self.active))
        self.t += self.dt
        for rid in list(self.active):
            self.active[rid][0] -= 1
            if self.active[rid][0] == 0:
                t_arr = self.active.pop(rid)[1]
                self.done.append(rid)
                self.finished[rid] = (t_arr, self.t)
        return len(self.active)

    def poll(self):
        out, self.done = self.done, []
        return out

    def result(self, rid):
        from types import SimpleNamespace
        t_arr, t_done = self.finished[rid]
        return SimpleNamespace(done=t_done, latency=t_done - t_arr)

    def drain(self):
        pass


def test_replay_steps_while_requests_arrive(monkeypatch):
    """A request is served from the first step after its arrival, not held
    back until the rest of the trace has arrived: with arrivals 10 steps
    apart and 3 evaluations each, no batch ever holds two requests, and each
    request's latency is its own 3 steps."""
    from paper_2207_14276_amd import serve
    fake = _FakeServer(dt=1.0)
    monkeypatch.setattr(serve.time, "sleep", lambda s: setattr(fake, "t", fake.t + s))
    arrivals = [(10.0 * q, 3) for q in range(5)]
    rep = serve.replay(fake, arrivals)
    assert len(rep.results) == 5
    assert all(len(b) == 1 for b in fake.batches)
    assert len(fake.batches) == 15
    np.testing.assert_allclose(rep.latencies(), 3.0)


def test_replay_joins_arrivals_into_running_batch(monkeypatch):
    """Requests arriving while others are in flight join the next step
    (continuous batching), and the replay runs until the last one is done."""
    from paper_2207_14276_amd import serve
    fake = _FakeServer(dt=1.0)
    monkeypatch.setattr(serve.time, "sleep", lambda s: setattr(fake, "t", fake.t + s))
    arrivals = [(0.0, 4), (1.5, 4), (2.5, 1)]
    rep = serve.replay(fake, arrivals)
    assert fake.batches[0] == [0]
    assert fake.batches[2] == [0, 1]
    assert fake.batches[3] == [0, 1, 2]
    assert sorted(rep.results) == [0, 1, 2]
    assert rep.wall == pytest.approx(max(r.done for r in rep.results.values()))


def test_failed_request_stops_alone():
    """A request that fails mid-flight leaves the flight and frees its slots
    for the queue; the others run all their steps; a failed or queued
    request cannot be failed (again)."""
    s = Scheduler(slots=100, max_batch_atoms=100)
    for rid, n in enumerate([40, 30, 30, 50]):
        s.submit(rid, n, 4, 0.0)
    assert [r for r, _ in s.admit(0.0)] == [0, 1, 2]
    with pytest.raises(NNPError):
        s.fail(3, 0.5)               # still queued
    s.launch()
    s.fail(1, 1.0)                   # stops after one launched step
    with pytest.raises(NNPError):
        s.fail(1, 1.5)
    assert s.info()["active"] == 2 and s.info()["free_slots"] == 30
    assert s.admit(1.0) == []        # 50 atoms: the 30 freed slots are not enough
    for _ in range(3):
        items = s.launch()
        assert sorted(it[0] for it in items) == [0, 2]
    assert s.info()["free_slots"] == 100
    assert [r for r, _ in s.admit(2.0)] == [3]
    assert s.job(1)["done"] == 1.0
