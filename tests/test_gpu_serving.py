"""Device-resident neighbour lists and the native continuous-batching
server, on the GPU through the C ABI.

Persistent lists (built with rc + skin, reused until an atom moved more than
skin/2) must give the results of fresh lists at every step of a random walk;
a request served inside a changing mix must give the same per-step results
as when served alone, and those match the oracle at the float32 tolerances;
memory and batch budgets make requests wait without changing any result.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import BF16_E_PER_ATOM, BF16_F, FP32_E_ATOM, FP32_F, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spec():
    return synth.make_model(0)


@pytest.fixture(scope="module")
def m32(spec):
    from paper_2207_14276_amd import NNPModel
    return NNPModel(spec, "fp32")


@pytest.fixture(scope="module")
def m16(spec):
    from paper_2207_14276_amd import NNPModel
    return NNPModel(spec, "bf16")


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


def test_pool_rows_follow_cutoff_box_and_size(m32):
    """A pool records what each system's rows were built for (box, list
    cutoff = model cutoff + skin, atom count): the same slots used by a model
    of a larger cutoff, or with the box changed, or by a system of another
    size, rebuild instead of reusing rows built for the old one.  Each result
    matches a fresh list's at the pool tolerances."""
    from paper_2207_14276_amd import NeighborPool, NNPModel
    dp = NNPModel(synth.make_dp_model(0), "fp32")  # cutoff 6.0 A (the ANI model's: 5.1 A)
    pool = NeighborPool(m32, slots=600, capacity=320, skin=0.5)

    def check(model, system, rebuild, expect_build):
        b = synth.make_batch([system])
        c = torch.as_tensor(b.coords, device="cuda")
        sp = torch.as_tensor(b.species, device="cuda")
        before = pool.builds()
        pool.model = model
        r = pool.energy_forces(c, sp, b.boxes, b.offsets, [0], [rebuild])
        ref = model.energy_forces(c, sp, b.boxes, b.offsets, check=True)
        torch.cuda.synchronize()
        de = float((r.energy - ref.energy).abs().max()) / system.n
        df = float((r.forces - ref.forces).abs().max())
        log(f"[pool record] n={system.n} box={system.box[0]:.2f} builds +{pool.builds() - before} "
            f"|dE|/N={de:.2e} |dF|={df:.2e}")
        assert pool.builds() == before + (1 if expect_build else 0)
        assert de <= 1e-6 and df <= 1e-5

    w = synth.water_box(60, seed=3)
    check(m32, w, 1, True)                       # first use of the slots
    check(m32, w, 0, False)                      # unchanged: the rows are reused
    check(dp, w, 0, True)                        # larger cutoff: rebuilt
    scaled = synth.System(w.coords * 1.04, w.species, w.box * 1.04)
    check(dp, scaled, 0, True)                   # box changed: rebuilt
    check(m32, synth.water_box(50, seed=4), 0, True)  # another system in the slots: rebuilt
    pool.model = m32
    pool.close()
    dp.close()


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


def _requests(n, seed, nmin=20, nmax=400, steps=6, sigma=0.01):
    from paper_2207_14276_amd.serve import Request
    rng = np.random.default_rng(seed)
    reqs = []
    for rid in range(n):
        size = int(rng.integers(nmin, nmax))
        if rid % 2 == 0:
            s = synth.water_box(max(1, size // 3), seed=1000 + rid)
        else:
            s = synth.random_solute(np.random.default_rng(2000 + rid), size,
                                    1.2 * size ** (1 / 3), synth.CONFIG2_PROBS)
        reqs.append(Request(s.coords, s.species, s.box, steps, sigma, seed=3000 + rid))
    return reqs


def _server(model, **kw):
    from paper_2207_14276_amd.serve import Server
    # dense solutes reach ~550 neighbours inside rc + skin
    opts = dict(slots=20000, capacity=640, skin=1.0)
    opts.update(kw)
    return Server(model, **opts)


def _run(model, reqs, spacing=0.0, **kw):
    from paper_2207_14276_amd.serve import replay
    srv = _server(model, **kw)
    rep = replay(srv, [(k * spacing, r) for k, r in enumerate(reqs)])
    stats = srv.stats()
    srv.close()
    return rep, stats


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_served_alone_equals_served_in_mix(m32, m16, oracle_lib, spec, prec):
    """Served in a changing mix or alone, a request gives the same walk, the
    same energies and the same forces, bit for bit;
    its last step matches the oracle at the tolerances of the precision form
    the server runs (float32, or bfloat16 dense layers as benchmarked)."""
    model = m32 if prec == "fp32" else m16
    e_tol, f_tol = (FP32_E_ATOM, FP32_F) if prec == "fp32" else (BF16_E_PER_ATOM, BF16_F)
    reqs = _requests(10, seed=5)
    # staggered arrivals: the mix around the tracked requests changes every few steps
    mixed, _ = _run(model, reqs, spacing=0.002)
    assert len(mixed.results) == 10
    for rid in (3, 6):
        alone, _ = _run(model, [reqs[rid]])
        a, m = alone.results[0], mixed.results[rid]
        assert np.array_equal(a.coords, m.coords)        # the client's walk is the same
        de = float(np.abs(a.energies - m.energies).max())
        df = float(np.abs(a.forces - m.forces).max())
        log(f"[alone-vs-mix {prec} rid={rid}] max|dE|={de:.3e} max|dF|={df:.3e}")
        # bit for bit: a row's dense-layer results do not depend on its tile,
        # force sums are integer (fixed point), reductions have a fixed order
        assert de == 0.0
        assert df == 0.0
        # the last step's results match the oracle at the coordinates evaluated
        om = oracle_lib.OracleModel(spec)
        E, ea, F, _ = oracle_lib.energy_forces(a.coords, reqs[rid].species, reqs[rid].box, om)
        de = abs(float(a.energies[-1]) - E) / reqs[rid].n_atoms
        df = float(np.abs(a.forces - F).max())
        log(f"[served vs oracle {prec} rid={rid}] |dE|/N={de:.3e} max|dF|={df:.3e}")
        assert de <= e_tol
        assert df <= f_tol


def test_server_drains_a_burst(m32):
    reqs = _requests(24, seed=9, nmin=20, nmax=600, steps=5)
    rep, st = _run(m32, reqs, spacing=0.0005)
    lat = rep.latencies()
    assert len(lat) == 24 and np.all(lat > 0)
    log(f"[serve burst] {st.atom_evals / rep.wall:.3e} atom-evals/s, iterations={st.iterations}, "
        f"p50={np.percentile(lat, 50) * 1e3:.2f} ms p99={np.percentile(lat, 99) * 1e3:.2f} ms, "
        f"list builds={st.list_builds}")
    assert st.atom_evals == sum(r.n_atoms * r.n_steps for r in reqs)
    # sigma = 0.01 A over 5 steps never moves an atom skin/2: one build per request
    assert st.list_builds == 24
    for r in rep.results.values():
        assert r.admitted >= r.arrival - 1e-9 and r.done > r.admitted


def test_batch_budget_queues_without_changing_results(m32):
    reqs = _requests(8, seed=21, nmin=100, nmax=250, steps=4)
    free, _ = _run(m32, reqs)
    tight, st = _run(m32, reqs, max_batch_atoms=300)
    log(f"[batch budget 300] iterations={st.iterations} max batch seen={st.max_batch_seen}")
    assert st.max_batch_atoms == 300 and st.max_batch_seen <= 300
    assert st.iterations > 4       # the requests could not all run side by side
    for rid in range(8):
        a, b = free.results[rid], tight.results[rid]
        assert np.array_equal(a.coords, b.coords)
        assert np.abs(a.energies - b.energies).max() <= 1e-9 * reqs[rid].n_atoms + 1e-12
        assert np.abs(a.forces - b.forces).max() <= 1e-5


def test_memory_budget_bounds_the_batch(spec):
    from paper_2207_14276_amd import NNPError, NNPModel
    from paper_2207_14276_amd.serve import replay
    # a fresh model: the budget covers the memory the server adds, and a model
    # that already holds a large workspace would need none
    model = NNPModel(spec, "fp32")
    budget = 64 << 20
    srv = _server(model, slots=4000, hbm_budget=budget)
    st = srv.stats()
    log(f"[hbm budget 64 MiB] batch budget={st.max_batch_atoms} atoms, granted={st.device_bytes} B")
    assert 0 < st.max_batch_atoms < 4000
    assert st.device_bytes <= budget
    big = _requests(1, seed=3, nmin=3000, nmax=3001)[0]
    if big.n_atoms > st.max_batch_atoms:
        with pytest.raises(NNPError):
            srv.submit(big)
    small = [r for r in _requests(12, seed=4, nmin=50, nmax=300, steps=3)
             if r.n_atoms <= st.max_batch_atoms]
    rep = replay(srv, [(0.0, r) for r in small])
    assert len(rep.results) == len(small)
    assert srv.stats().max_batch_seen <= st.max_batch_atoms
    srv.close()
    model.close()


def test_random_walk_statistics(m32):
    from paper_2207_14276_amd.serve import Request
    s = synth.water_box(300, seed=77)
    sigma, steps = 0.01, 9
    rep, _ = _run(m32, [Request(s.coords, s.species, s.box, steps, sigma, seed=123)])
    d = (rep.results[0].coords.astype(np.float64) - s.coords).ravel()
    var = d.var() / (sigma ** 2 * (steps - 1))
    log(f"[walk] n={d.size} mean={d.mean():.2e} var ratio={var:.3f}")
    assert abs(d.mean()) < 5 * sigma * np.sqrt(steps - 1) / np.sqrt(d.size)
    assert 0.9 < var < 1.1


def test_capacity_overflow_is_reported(m32):
    """Every request of this server overflows a 16-entry capacity: each one
    stops alone with NNP_ECAPACITY, the server drains, and the model's flags
    are clear again once the server is gone."""
    from paper_2207_14276_amd import _native as nat
    rep, _ = _run(m32, _requests(2, seed=5, steps=2), capacity=16)
    assert len(rep.results) == 2
    for r in rep.results.values():
        log(f"[overflow] request {r.rid}: {r.message}")
        assert r.error == nat.NNP_ECAPACITY
        assert "capacity of 16" in r.message
    m32.status()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_overflowing_request_fails_alone(m32, m16, oracle_lib, spec, prec):
    """A dense 300-atom solute (~550 neighbours inside rc + skin) among small
    requests on a server of capacity 128: it stops with NNP_ECAPACITY and
    every other request runs all its steps with the results it gets when
    served alone (bit for bit: integer force sums), its last step matching
    the oracle."""
    from paper_2207_14276_amd import _native as nat
    from paper_2207_14276_amd.serve import Request
    model = m32 if prec == "fp32" else m16
    e_tol, f_tol = (FP32_E_ATOM, FP32_F) if prec == "fp32" else (BF16_E_PER_ATOM, BF16_F)
    dense = synth.random_solute(np.random.default_rng(300), 300, 1.2 * 300 ** (1 / 3), synth.CONFIG2_PROBS)
    small = [synth.random_solute(np.random.default_rng(61), 60, 1.2 * 60 ** (1 / 3), synth.CONFIG2_PROBS),
             synth.water_box(30, seed=62), None,
             synth.random_solute(np.random.default_rng(63), 80, 1.2 * 80 ** (1 / 3), synth.CONFIG2_PROBS),
             synth.water_box(20, seed=64)]
    systems = [dense if x is None else x for x in small]
    reqs = [Request(x.coords, x.species, x.box, 4, 0.01, seed=700 + k) for k, x in enumerate(systems)]
    mixed, _ = _run(model, reqs, spacing=0.001, capacity=128)
    assert len(mixed.results) == 5
    bad = mixed.results[2]
    log(f"[fails alone {prec}] {bad.message}")
    assert bad.error == nat.NNP_ECAPACITY
    om = oracle_lib.OracleModel(spec)
    for rid in (0, 1, 3, 4):
        m = mixed.results[rid]
        assert m.error == 0
        alone, _ = _run(model, [reqs[rid]], capacity=128)
        a = alone.results[0]
        assert np.array_equal(a.coords, m.coords)
        assert np.array_equal(a.energies, m.energies)
        assert np.array_equal(a.forces, m.forces)
        E, _, F, _ = oracle_lib.energy_forces(m.coords, reqs[rid].species, reqs[rid].box, om, virial=False)
        de = abs(float(m.energies[-1]) - E) / reqs[rid].n_atoms
        df = float(np.abs(m.forces - F).max())
        log(f"[fails alone {prec}] request {rid}: |dE|/N={de:.3e} max|dF|={df:.3e}")
        assert de <= e_tol and df <= f_tol
    model.status()


def test_bad_species_refused_at_submission(m32):
    from paper_2207_14276_amd import NNPError
    from paper_2207_14276_amd.serve import Request
    srv = _server(m32, slots=2000)
    s = synth.water_box(5, seed=3)
    sp = s.species.copy()
    sp[4] = 9
    with pytest.raises(NNPError, match="ESPECIES"):
        srv.submit(Request(s.coords, sp, s.box, 2, 0.01, seed=1))
    srv.close()
    m32.status()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_graph_replay_equals_direct_launches(m32, m16, prec):
    """The same requests served with every iteration replayed from a graph
    recorded once per capacity bucket, and with every kernel launched
    directly: identical walks, energies and forces, bit for bit (results do
    not depend on the mix, so the two runs' different batching does not
    matter); most iterations replay a graph recorded earlier."""
    model = m32 if prec == "fp32" else m16
    reqs = _requests(16, seed=21, nmin=20, nmax=900, steps=8)
    g, sg = _run(model, reqs, spacing=0.001, use_graphs=True)
    d, sd = _run(model, reqs, spacing=0.001, use_graphs=False)
    log(f"[graphs {prec}] iterations {sg.iterations} (direct run: {sd.iterations}), "
        f"graphs recorded {sg.graph_captures}, replays {sg.graph_replays}; host time per iteration "
        f"{sg.host_launch_s / max(sg.iterations, 1) * 1e6:.0f} us with graphs, "
        f"{sd.host_launch_s / max(sd.iterations, 1) * 1e6:.0f} us direct")
    assert len(g.results) == len(d.results) == len(reqs)
    for rid in range(len(reqs)):
        a, b = g.results[rid], d.results[rid]
        assert a.error == 0 and b.error == 0
        assert np.array_equal(a.coords, b.coords)
        assert np.array_equal(a.energies, b.energies)
        assert np.array_equal(a.forces, b.forces)
    assert sg.graph_replays == sg.iterations
    assert 1 <= sg.graph_captures < sg.iterations
    assert sd.graph_replays == 0 and sd.graph_captures == 0
