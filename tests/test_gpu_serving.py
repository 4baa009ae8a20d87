"""Device-resident neighbour lists and the continuous-batching server, on the
GPU through the C ABI.

Persistent lists (built with rc + skin, reused until an atom moved more than
skin/2) must give the results of fresh lists at every step of a random walk;
a request served inside a changing mix must give the same per-step results
as when served alone, and those match the oracle at the float32 tolerances.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import FP32_E_ATOM, FP32_F, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spec():
    return synth.make_model(0)


@pytest.fixture(scope="module")
def m32(spec):
    from paper_2207_14276_amd import NNPModel
    return NNPModel(spec, "fp32")


def _walk(batch, steps, sigma, seed):
    rng = np.random.default_rng(seed)
    x = batch.coords.astype(np.float32)
    for _ in range(steps):
        yield x
        x = (x + rng.normal(0.0, sigma, size=x.shape)).astype(np.float32)


def _systems():
    return synth.make_batch([synth.water_box(100, seed=11),
                             synth.ragged_solutes(1, seed=12, nmin=80, nmax=80).systems[0],
                             synth.water_box(7, seed=13)])


@pytest.mark.parametrize("sigma,expect_rebuilds", [(0.01, False), (0.15, True)])
def test_pool_lists_match_fresh_lists(m32, sigma, expect_rebuilds):
    from paper_2207_14276_amd import NeighborPool
    b = _systems()
    pool = NeighborPool(m32, slots=1000, capacity=256, skin=1.0)
    # systems placed in the pool away from their batch positions
    slots = np.array([500, 100, 900], np.int64)
    sp = torch.as_tensor(b.species, device="cuda")
    worst_e = worst_f = 0.0
    for step, x in enumerate(_walk(b, 12, sigma, seed=3)):
        c = torch.as_tensor(x, device="cuda")
        rb = np.ones(3, np.int32) if step == 0 else None
        r1 = pool.energy_forces(c, sp, b.boxes, b.offsets, slots, rb)
        r0 = m32.energy_forces(c, sp, b.boxes, b.offsets, check=True)
        torch.cuda.synchronize()
        n = np.diff(b.offsets)
        worst_e = max(worst_e, float(((r1.energy - r0.energy).abs().cpu().numpy() / n).max()))
        worst_f = max(worst_f, float((r1.forces - r0.forces).abs().max()))
    builds = pool.builds()
    log(f"[pool sigma={sigma}] max|dE|/N={worst_e:.3e} max|dF|={worst_f:.3e} builds={builds}")
    assert worst_e <= 1e-6
    assert worst_f <= 1e-5
    if expect_rebuilds:
        assert builds > 3
    else:
        assert builds == 3
    m32.status()


def test_pool_rejects_bad_slot_ranges(m32):
    from paper_2207_14276_amd import NeighborPool, NNPError
    b = _systems()
    pool = NeighborPool(m32, slots=400, capacity=64, skin=1.0)
    c = torch.as_tensor(b.coords, device="cuda")
    sp = torch.as_tensor(b.species, device="cuda")
    with pytest.raises(NNPError):   # overlapping ranges
        pool.energy_forces(c, sp, b.boxes, b.offsets, [0, 10, 200], [1, 1, 1])
    with pytest.raises(NNPError):   # beyond the pool
        pool.energy_forces(c, sp, b.boxes, b.offsets, [0, 300, 390], [1, 1, 1])


def _requests(n, seed, nmin=20, nmax=400, steps=6, record=()):
    from paper_2207_14276_amd.serve import Job, SystemPayload
    rng = np.random.default_rng(seed)
    jobs = []
    for rid in range(n):
        size = int(rng.integers(nmin, nmax))
        if rid % 2 == 0:
            s = synth.water_box(max(1, size // 3), seed=1000 + rid)
        else:
            s = synth.random_solute(np.random.default_rng(2000 + rid), size,
                                    1.2 * size ** (1 / 3), synth.CONFIG2_PROBS)
        p = SystemPayload(s.coords, s.species, s.box, seed=3000 + rid, sigma=0.01,
                          record=rid in record)
        jobs.append(Job(rid, s.n, steps, 0.0, payload=p))
    return jobs


def _run(model, jobs, spacing=0.0):
    from paper_2207_14276_amd.serve import GpuExecutor, Scheduler, serve
    # dense solutes reach ~550 neighbours inside rc + skin
    ex = GpuExecutor(model, slots=20000, capacity=640, skin=1.0)
    sched = Scheduler(slots=20000, max_batch_atoms=20000)
    arrivals = [(k * spacing, j) for k, j in enumerate(jobs)]
    wall = serve(ex, sched, arrivals, sync=torch.cuda.synchronize)
    return sched, ex, wall


def test_served_alone_equals_served_in_mix(m32, oracle_lib, spec):
    jobs = _requests(10, seed=5, record=(3, 6))
    # staggered arrivals: the mix around the tracked jobs changes every few steps
    sched, ex, wall = _run(m32, jobs, spacing=0.002)
    assert len(sched.finished) == 10
    mixed = {j.rid: j.payload.trace for j in jobs if j.rid in (3, 6)}
    for rid in (3, 6):
        alone = _requests(10, seed=5, record=(rid,))[rid]
        _run(m32, [alone])
        t_mix, t_alone = mixed[rid], alone.payload.trace
        assert len(t_mix) == len(t_alone) == alone.n_steps
        worst_e = worst_f = 0.0
        for (cm, em, fm), (ca, ea, fa) in zip(t_mix, t_alone):
            assert torch.equal(cm, ca)          # the client's walk is the same
            worst_e = max(worst_e, abs(float(em[0]) - float(ea[0])))
            worst_f = max(worst_f, float((fm - fa).abs().max()))
        log(f"[alone-vs-mix rid={rid}] max|dE|={worst_e:.3e} max|dF|={worst_f:.3e}")
        assert worst_e <= 1e-9 * alone.n_atoms + 1e-12
        assert worst_f <= 1e-5
        # and the served result matches the oracle on the last step's coordinates
        p = alone.payload
        x, e, f = t_alone[-1]
        om = oracle_lib.OracleModel(spec)
        E, ea, F, _ = oracle_lib.energy_forces(x.cpu().numpy(), p.species, p.box, om)
        de = abs(float(e[0]) - E) / alone.n_atoms
        df = float(np.abs(f.cpu().numpy() - F).max())
        log(f"[served vs oracle rid={rid}] |dE|/N={de:.3e} max|dF|={df:.3e}")
        assert de <= FP32_E_ATOM
        assert df <= FP32_F


def test_server_drains_a_burst(m32):
    jobs = _requests(24, seed=9, nmin=20, nmax=600, steps=5)
    sched, ex, wall = _run(m32, jobs, spacing=0.0005)
    lat = sched.latencies()
    assert len(lat) == 24
    log(f"[serve burst] {sched.atom_evals / wall:.3e} atom-evals/s, iterations={sched.iterations}, "
        f"p50={np.percentile(lat, 50) * 1e3:.2f} ms p99={np.percentile(lat, 99) * 1e3:.2f} ms, "
        f"list builds={ex.builds()}")
    # every job was admitted at once (budget large enough): one build each
    assert ex.builds() == 24
