"""Host logic of the serving loop, against a mock executor (no GPU):
slot allocation, first-come first-served admission under slot and batch
budgets, continuous joining of new requests, step accounting and latencies."""
import numpy as np
import pytest

from paper_2207_14276_amd.serve import Job, Scheduler, SlotAllocator, serve


def test_slot_allocator_first_fit_and_merge():
    a = SlotAllocator(100)
    s1 = a.alloc(30)
    s2 = a.alloc(30)
    s3 = a.alloc(30)
    assert (s1, s2, s3) == (0, 30, 60)
    assert a.alloc(20) is None            # only 10 free
    a.release(s2, 30)
    assert a.alloc(35) is None            # the hole is 30 wide
    assert a.alloc(25) == 30
    a.release(s1, 30)
    a.release(30, 25)
    assert a.free == [(0, 60), (90, 10)]  # merged
    assert a.free_slots == 70


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class MockExecutor:
    """Stands in for the GPU: each evaluation takes `dt` of fake time."""

    def __init__(self, clock, dt=1.0):
        self.clock, self.dt = clock, dt
        self.batches = []
        self.admitted = []

    def admit(self, job):
        self.admitted.append(job.rid)

    def evaluate(self, batch):
        self.batches.append([j.rid for j in batch])
        self.clock.t += self.dt

    def advance(self, batch, finished):
        pass


def test_fcfs_admission_respects_both_budgets():
    clk = FakeClock()
    s = Scheduler(slots=100, max_batch_atoms=80, clock=clk)
    for rid, n in enumerate([50, 40, 20, 10]):
        s.submit(Job(rid, n, n_steps=2, arrival=0.0))
    got = s.admit()
    # 50 fits; 40 would exceed the 80-atom batch budget; 20 and 10 wait behind it
    assert [j.rid for j in got] == [0]
    s.complete(s.batch(), 1.0)
    assert s.admit() == []
    s.complete(s.batch(), 2.0)           # job 0 finishes after 2 steps
    assert [j.rid for j in s.finished] == [0]
    assert [j.rid for j in s.admit()] == [1, 2, 3]


def test_oversized_request_is_rejected():
    s = Scheduler(slots=100, max_batch_atoms=50)
    with pytest.raises(ValueError):
        s.submit(Job(0, 60, 1, 0.0))


def test_continuous_batching_joins_new_requests_mid_flight():
    clk = FakeClock()
    ex = MockExecutor(clk, dt=1.0)
    s = Scheduler(slots=1000, max_batch_atoms=1000, clock=clk)
    arrivals = [(0.0, Job(0, 10, 5, 0.0)), (2.5, Job(1, 20, 2, 0.0)), (2.5, Job(2, 5, 1, 0.0))]
    serve(ex, s, arrivals, clock=clk)
    # job 0 runs alone for three iterations, then 1 and 2 join the batch
    assert ex.batches[:3] == [[0], [0], [0]]
    assert ex.batches[3] == [0, 1, 2]
    assert ex.batches[4] == [0, 1]
    assert len(s.finished) == 3
    lat = {j.rid: j.done_time - j.arrival for j in s.finished}
    assert lat[0] == pytest.approx(5.0)
    assert lat[2] == pytest.approx(1.5)
    assert s.atom_evals == 10 * 5 + 20 * 2 + 5 * 1


def test_queue_waits_for_slots_then_drains():
    clk = FakeClock()
    ex = MockExecutor(clk, dt=1.0)
    s = Scheduler(slots=30, max_batch_atoms=1000, clock=clk)
    arrivals = [(0.0, Job(k, 20, 3, 0.0)) for k in range(4)]
    serve(ex, s, arrivals, clock=clk)
    # one 20-atom job fits the 30 slots at a time: strictly sequential, none lost
    assert all(len(b) == 1 for b in ex.batches)
    assert sorted(j.rid for j in s.finished) == [0, 1, 2, 3]
    lat = s.latencies()
    np.testing.assert_allclose(sorted(lat), [3, 6, 9, 12])
