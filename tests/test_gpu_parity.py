"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: neighbour lists are integer work and must match the brute-force
oracle exactly (entries within 1e-5 A of the cutoff, where float32 and
float64 distances may decide differently, are listed and excluded); the
float32 path holds |dE_i| <= 1e-5 kcal/mol per atom, |dE_s|/N_s <= 1e-5 and
|dF| <= 1e-3 kcal/mol/A; the bfloat16 dense-layer path holds |dE_s|/N_s <=
1e-2 and |dF| <= 5e-2.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import (BF16_E_PER_ATOM, BF16_F, FP32_E_ATOM, FP32_F, log, run_gpu, to_dev,
                            virial_bound)

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


@pytest.fixture(scope="module")
def om(oracle_lib, spec):
    return oracle_lib.OracleModel(spec)


def small_systems():
    return {
        "cluster24": synth.make_batch([synth.config0()]),
        "water8_small_box": synth.make_batch([synth.water_box(8, seed=5)]),
        "water2_tiny_box": synth.make_batch([synth.water_box(2, seed=6)]),
        # one cell of ~4.5 A with 9 atoms: two images deep in every direction
        "water3_tiny_box": synth.make_batch([synth.water_box(3, seed=7)]),
        "ragged16": synth.ragged_solutes(16, seed=12),
        "water667": synth.make_batch([synth.config1()]),
    }


SYSTEMS = small_systems()


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_neighbour_lists_match_brute_force(m32, oracle_lib, name):
    b = SYSTEMS[name]
    c, s, bx, o = to_dev(b)
    cap = 256
    m32.reserve(b.n_atoms, b.n_systems, cap)
    cnt, ent = m32.neighbors(c, s, bx, o, capacity=cap)
    cnt = cnt.cpu().numpy()
    ent = ent.cpu().numpy()
    rc = m32.spec.aev["rc_rad"]
    n_edge = 0
    for k in range(b.n_systems):
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        sysc = b.coords[a:e].astype(np.float64)
        for i in range(a, e):
            gpu = {(int(r[0]) - a, (int(r[1]), int(r[2]), int(r[3]))) for r in ent[i, :cnt[i]]}
            assert len(gpu) == cnt[i]
            ref = set(oracle_lib.neighbours(b.coords[a:e], b.boxes[k], rc, i - a))
            diff = gpu ^ ref
            for j, img in diff:
                d = sysc[j] + np.array(img) * b.boxes[k].astype(np.float64) - sysc[i - a]
                assert abs(np.linalg.norm(d) - rc) < 1e-5 * rc, (name, i, j, img, np.linalg.norm(d))
                n_edge += 1
    log(f"[nbr] {name}: atoms={b.n_atoms} max_count={cnt.max()} boundary_entries={n_edge}")


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_aev_matches_oracle(m32, oracle_lib, name):
    b = SYSTEMS[name]
    c, s, bx, o = to_dev(b)
    G = m32.aev(c, s, bx, o).cpu().numpy().astype(np.float64)
    worst = 0.0
    for k in range(b.n_systems):
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        ref = oracle_lib.aev(b.coords[a:e], b.species[a:e], b.boxes[k], m32.spec.aev)
        err = np.abs(G[a:e] - ref) / (1.0 + np.abs(ref))
        worst = max(worst, float(err.max()))
    log(f"[aev] {name}: max |dG|/(1+|G|) = {worst:.3e}")
    # float32 evaluation of sums of O(100) terms, each with ~1e-6 relative error
    assert worst < 2e-5


def test_aev_rows_rewritten_whole(spec, oracle_lib):
    """Every call rewrites each feature row whole: after a batch with many
    species, a water box (H and O only) reuses the same rows.  Its features
    match the oracle with exact zeros in the blocks of species pairs that
    have no pair around a centre, and its energies equal those of a fresh
    model bit for bit (forces to float32 rounding), in float32 and in
    bfloat16 feature rows."""
    from paper_2207_14276_amd import NNPModel
    first = synth.ragged_solutes(16, seed=12)
    second = synth.make_batch([synth.config1()])
    ref = oracle_lib.aev(second.coords, second.species, second.boxes[0], spec.aev)
    zero_cols = np.all(ref == 0.0, axis=0)
    assert zero_cols.sum() > 0
    m = NNPModel(spec, "fp32")
    c, s, bx, o = to_dev(first)
    m.aev(c, s, bx, o)
    c, s, bx, o = to_dev(second)
    G = m.aev(c, s, bx, o).cpu().numpy().astype(np.float64)
    m.close()
    err = np.abs(G - ref) / (1.0 + np.abs(ref))
    log(f"[aev reuse] max |dG|/(1+|G|) = {err.max():.3e}, zero columns = {int(zero_cols.sum())}")
    assert err.max() < 2e-5
    assert np.all(G[:, zero_cols] == 0.0)
    for prec in ("fp32", "bf16"):
        used, fresh = NNPModel(spec, prec), NNPModel(spec, prec)
        run_gpu(used, first)
        a, b = run_gpu(used, second), run_gpu(fresh, second)
        used.close()
        fresh.close()
        # energies: deterministic reduction; forces: 64-bit fixed-point sums,
        # the same whatever order the centres add in
        assert np.array_equal(a["energy"], b["energy"]), prec
        assert np.array_equal(a["forces"], b["forces"]), prec


def _check_energy_forces(model, oracle_lib, om, b, systems, e_atom_tol, e_sys_tol, f_tol, label):
    gpu = run_gpu(model, b)
    ora = oracle_lib.batch_energy_forces(b, om, systems=systems)
    worst_ea = worst_es = worst_f = worst_w = 0.0
    worst_wr = 0.0   # virial error as a fraction of its derived bound
    for q, k in enumerate(systems):
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        n = e - a
        if n == 0:
            assert gpu["energy"][k] == 0.0
            continue
        worst_ea = max(worst_ea, float(np.abs(gpu["e_atom"][a:e] - ora["e_atom"][q]).max()))
        worst_es = max(worst_es, abs(gpu["energy"][k] - ora["energy"][q]) / n)
        worst_f = max(worst_f, float(np.abs(gpu["forces"][a:e] - ora["forces"][q]).max()))
        dw = float(np.abs(gpu["virial"][k] - ora["virial"][q]).max())
        worst_w = max(worst_w, dw / n)
        bound = virial_bound(b.coords[a:e], b.boxes[k], gpu["forces"][a:e], ora["forces"][q],
                             w_ref=ora["virial"][q])
        worst_wr = max(worst_wr, dw / bound)
    log(f"[{label}] max|dE_i|={worst_ea:.3e} max|dE_s|/N={worst_es:.3e} "
        f"max|dF|={worst_f:.3e} max|dW|/N={worst_w:.3e} max|dW|/bound={worst_wr:.3f}")
    if e_atom_tol is not None:
        assert worst_ea <= e_atom_tol
    assert worst_es <= e_sys_tol
    assert worst_f <= f_tol
    # the virial error follows from the force error (virial_bound)
    assert worst_wr <= 1.0
    return gpu, ora


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_fp32_energy_forces_match_oracle(m32, oracle_lib, om, name):
    b = SYSTEMS[name]
    _check_energy_forces(m32, oracle_lib, om, b, list(range(b.n_systems)), FP32_E_ATOM, FP32_E_ATOM,
                         FP32_F, f"fp32 {name}")


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_bf16_energy_forces_match_oracle(m16, oracle_lib, om, name):
    b = SYSTEMS[name]
    _check_energy_forces(m16, oracle_lib, om, b, list(range(b.n_systems)), None, BF16_E_PER_ATOM,
                         BF16_F, f"bf16 {name}")


def test_ragged_batch_512_sampled_systems(m32, m16, oracle_lib, om):
    """The full 512-solute batch in one call; 24 seeded systems checked,
    including the smallest and the largest."""
    b = synth.config2()
    sizes = np.diff(b.offsets)
    rng = np.random.default_rng(0)
    pick = sorted(set(rng.choice(b.n_systems, 22, replace=False).tolist()
                      + [int(sizes.argmin()), int(sizes.argmax())]))
    _check_energy_forces(m32, oracle_lib, om, b, pick, FP32_E_ATOM, FP32_E_ATOM, FP32_F, "fp32 ragged512")
    _check_energy_forces(m16, oracle_lib, om, b, pick, None, BF16_E_PER_ATOM, BF16_F, "bf16 ragged512")


def test_ensemble_mean(oracle_lib):
    from paper_2207_14276_amd import NNPModel
    spec = synth.make_model(7, n_ensemble=3)
    m = NNPModel(spec, "fp32")
    om = oracle_lib.OracleModel(spec)
    for name in ("cluster24", "water8_small_box", "ragged16"):
        b = SYSTEMS[name]
        _check_energy_forces(m, oracle_lib, om, b, list(range(b.n_systems)), FP32_E_ATOM,
                             FP32_E_ATOM, FP32_F, f"fp32 ensemble3 {name}")


@pytest.mark.parametrize("hidden", [(72, 40), (96, 64), (128, 96, 64, 32)],
                         ids=["unfused-widths-72-40", "chain-1-layer", "chain-3-layers"])
def test_bf16_network_shapes(oracle_lib, hidden):
    """bfloat16 networks of other shapes, 2 members: hidden widths that are
    not multiples of 32 run the layer-by-layer GEMMs (register-staged tiles,
    element output layer); the others run the fused hidden-layer chain with
    one and with three layers after the first."""
    from paper_2207_14276_amd import NNPModel
    spec = synth.make_model(11, n_ensemble=2, hidden=[hidden] * 7)
    m = NNPModel(spec, "bf16")
    om = oracle_lib.OracleModel(spec)
    for name in ("cluster24", "water8_small_box", "ragged16"):
        b = SYSTEMS[name]
        _check_energy_forces(m, oracle_lib, om, b, list(range(b.n_systems)), None,
                             BF16_E_PER_ATOM, BF16_F, f"bf16 {hidden} {name}")


def test_linear_readout_model(oracle_lib):
    """Networks without hidden layers: energy linear in the AEV, so energy
    and force errors come from the AEV and its gradient alone."""
    from paper_2207_14276_amd import NNPModel
    spec = synth.linear_readout_model(3)
    m = NNPModel(spec, "fp32")
    om = oracle_lib.OracleModel(spec)
    for name in ("cluster24", "water667"):
        b = SYSTEMS[name]
        _check_energy_forces(m, oracle_lib, om, b, list(range(b.n_systems)), FP32_E_ATOM,
                             FP32_E_ATOM, FP32_F, f"fp32 linear {name}")


def test_forces_match_finite_differences(m32, oracle_lib, om):
    """Water box: GPU forces against central differences (h = 1e-4 A) of the
    oracle energy on 16 seeded atoms.  Moving atom t changes only the atomic
    energies of t and of centres with t inside the radial cutoff, so the
    difference is taken over those atoms."""
    s = synth.config1()
    b = synth.make_batch([s])
    gpu = run_gpu(m32, b, virial=False)
    rng = np.random.default_rng(16)
    rc = m32.spec.aev["rc_rad"]
    worst = 0.0
    h = 1e-4
    for t in rng.choice(s.n, 16, replace=False):
        centres = sorted({t} | {j for j, _ in oracle_lib.neighbours(s.coords, s.box, rc, int(t))})
        for a in range(3):
            es = []
            for sgn in (1, -1):
                x = s.coords.astype(np.float64).copy()
                x[t, a] += sgn * h
                e, _ = _sampled64(oracle_lib, om, x, s, centres)
                es.append(e.sum())
            fd = -(es[0] - es[1]) / (2 * h)
            worst = max(worst, abs(fd - gpu["forces"][t, a]))
    log(f"[fd] water667 16 atoms: max|F_gpu - F_fd| = {worst:.3e}")
    assert worst <= FP32_F


def _sampled64(oracle_lib, om, x64, s, targets):
    import ctypes as C
    lib = oracle_lib._load()
    x = np.ascontiguousarray(x64)
    sp = np.ascontiguousarray(s.species, np.int32)
    bx = np.ascontiguousarray(s.box.astype(np.float64))
    t = np.ascontiguousarray(targets, np.int32)
    e = np.zeros(len(t))
    f = np.zeros((len(t), 3))
    rc = lib.orc_sampled(s.n, oracle_lib._dp(x), oracle_lib._ip(sp), oracle_lib._dp(bx),
                         C.byref(om.struct), len(t), oracle_lib._ip(t), oracle_lib._dp(e),
                         oracle_lib._dp(f))
    assert rc == 0
    return e, f


def _protein_box_samples(s, n_protein=30000, per_group=16, seed=3):
    """Seeded atoms of the solvated-protein box in three groups: protein
    interior (more than 6 A inside the sphere), the protein/water interface
    (half protein atoms within 2.5 A of the sphere's surface, half waters
    within 4 A outside it) and bulk water (more than 8 A outside it)."""
    L = s.box.astype(np.float64)
    x = s.coords.astype(np.float64)
    r = np.linalg.norm(x - L / 2, axis=1)
    R = np.linalg.norm(x[:n_protein] - L / 2, axis=1).max()
    idx = np.arange(s.n)
    rng = np.random.default_rng(seed)
    draw = lambda v, k: np.sort(rng.choice(v, k, replace=False))
    h = per_group // 2
    return {"interior": draw(idx[(idx < n_protein) & (r < R - 6.0)], per_group),
            "interface": np.concatenate([draw(idx[(idx < n_protein) & (r > R - 2.5)], h),
                                         draw(idx[(idx >= n_protein) & (r < R + 4.0)], per_group - h)]),
            "water": draw(idx[(idx >= n_protein) & (r > R + 8.0)], per_group)}


def test_large_periodic_ensemble_sampled(oracle_lib):
    """~100k-atom periodic box with an ensemble of 8 networks, at full size in
    one call; atomic energies and forces of 48 seeded atoms (16 in the
    protein's interior, 16 at the protein/water interface, 16 in bulk water)
    against the oracle's local evaluation, plus the zero net force of the
    whole box."""
    from paper_2207_14276_amd import NNPModel
    spec = synth.make_model(3, n_ensemble=8)
    s = synth.config3()
    b = synth.make_batch([s])
    om = oracle_lib.OracleModel(spec)
    groups = _protein_box_samples(s)
    t = np.concatenate(list(groups.values()))
    e_ref, f_ref = oracle_lib.sampled(s.coords, s.species, s.box, om, t)
    for prec, e_tol, f_tol in (("fp32", FP32_E_ATOM, FP32_F), ("bf16", BF16_E_PER_ATOM, BF16_F)):
        m = NNPModel(spec, prec)
        gpu = run_gpu(m, b)
        de_all = np.abs(gpu["e_atom"][t] - e_ref)
        df_all = np.abs(gpu["forces"][t] - f_ref).max(1)
        net = float(np.abs(gpu["forces"].sum(0)).max())
        k = 0
        for g, v in groups.items():
            log(f"[{prec} protein100k ens8 {g}: {len(v)} atoms] max|dE_i|={de_all[k:k + len(v)].max():.3e} "
                f"max|dF|={df_all[k:k + len(v)].max():.3e}")
            k += len(v)
        log(f"[{prec} protein100k ens8] |sum F|={net:.3e}")
        assert float(de_all.max()) <= e_tol
        assert float(df_all.max()) <= f_tol
        assert net <= 1e-3 * np.sqrt(s.n) * max(1.0, np.abs(gpu["forces"]).max())
        m.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_alone_vs_mix(m32, m16, prec):
    """Each system gives the same result alone and inside a ragged batch, bit
    for bit: a row's dense-layer results do not depend on its tile, the AEV
    backward's force sums are integer (fixed point), and the energy
    reduction has a fixed order.  Also across repeated calls."""
    model = m32 if prec == "fp32" else m16
    b = synth.ragged_solutes(24, seed=33)
    mix = run_gpu(model, b)
    again = run_gpu(model, b)
    assert np.array_equal(mix["forces"], again["forces"])
    assert np.array_equal(mix["energy"], again["energy"])
    for k in range(0, 24, 5):
        one = synth.make_batch([b.systems[k]])
        alone = run_gpu(model, one)
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        de = abs(alone["energy"][0] - mix["energy"][k])
        df = float(np.abs(alone["forces"] - mix["forces"][a:e]).max())
        dw = float(np.abs(alone["virial"][0] - mix["virial"][k]).max())
        log(f"[alone-vs-mix {prec} system {k}] |dE|={de:.3e} max|dF|={df:.3e} max|dW|={dw:.3e}")
        assert de == 0.0
        assert df == 0.0
        assert dw == 0.0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_system_order_changes_no_result(m32, m16, prec):
    """The same systems in another order give the same per-system results,
    bit for bit: whatever the caller's order, the AEV kernels take the
    centres of a multi-system call largest system first, keep the force sums
    in that launch order and list the bucket rows in it."""
    model = m32 if prec == "fp32" else m16
    b = synth.ragged_solutes(40, seed=41)
    ref = run_gpu(model, b)
    perm = np.random.default_rng(5).permutation(40)
    pb = synth.make_batch([b.systems[k] for k in perm])
    got = run_gpu(model, pb)
    for q, k in enumerate(perm):
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        pa, pe = int(pb.offsets[q]), int(pb.offsets[q + 1])
        assert got["energy"][q] == ref["energy"][k], (q, k)
        assert np.array_equal(got["forces"][pa:pe], ref["forces"][a:e]), (q, k)
        assert np.array_equal(got["virial"][q], ref["virial"][k]), (q, k)
    log(f"[system order {prec}] 40 systems permuted: energies, forces and virials equal bit for bit")


def test_stage_timing_modes(m16):
    """Stage timing: every stage boundary, or only the two events around one
    stage (the others reported as not recorded); results unchanged."""
    b = synth.ragged_solutes(12, seed=7)
    ref = run_gpu(m16, b)
    m16.set_timing(True)
    got = run_gpu(m16, b)
    all_stages = m16.stage_timings()
    m16.set_timing(True, stage="aev_bwd")
    run_gpu(m16, b)
    run_gpu(m16, b)
    one = m16.stage_timings()
    m16.set_timing(False)
    log(f"[timing] all stages {all_stages}; aev_bwd alone {one}")
    assert list(all_stages) == list(m16.STAGES) and all(v >= 0.0 for v in all_stages.values())
    assert list(one) == ["aev_bwd"] and one["aev_bwd"] > 0.0
    assert np.array_equal(got["forces"], ref["forces"])


def test_edge_cases(m32, oracle_lib, om):
    """Empty systems, single atoms (no neighbours), one atom alone in a
    periodic box (self-images only), in one ragged batch."""
    lone = synth.System(np.array([[0.3, 0.2, 0.1]], np.float32), np.array([synth.C], np.int32),
                        np.zeros(3, np.float32))
    empty = synth.System(np.zeros((0, 3), np.float32), np.zeros(0, np.int32), np.zeros(3, np.float32))
    self_img = synth.System(np.array([[1.0, 1.0, 1.0]], np.float32), np.array([synth.O], np.int32),
                            np.array([3.1, 3.1, 3.1], np.float32))
    pair_img = synth.System(np.array([[0.5, 0.5, 0.5], [1.7, 0.9, 1.1]], np.float32),
                            np.array([synth.H, synth.N], np.int32), np.array([4.0, 3.0, 5.0], np.float32))
    b = synth.make_batch([empty, lone, synth.config0(), empty, self_img, pair_img, empty])
    _check_energy_forces(m32, oracle_lib, om, b, list(range(b.n_systems)), FP32_E_ATOM, FP32_E_ATOM,
                         FP32_F, "fp32 edge cases")


def test_bad_species_and_capacity_flags(spec):
    from paper_2207_14276_amd import NNPModel, NNPError
    from paper_2207_14276_amd import _native as nat
    m = NNPModel(spec, "fp32")
    b = synth.make_batch([synth.config0()])
    c, s, bx, o = to_dev(b)
    s_bad = s.clone()
    s_bad[3] = 9
    m.energy_forces(c, s_bad, bx, o)
    with pytest.raises(NNPError) as ei:
        m.status()
    assert ei.value.code == nat.NNP_ESPECIES
    # a capacity below the real neighbour count raises the overflow flag; the
    # checked call retries with a larger capacity and then matches
    w = synth.make_batch([synth.water_box(30, seed=2)])
    cw, sw, bw, ow = to_dev(w)
    m.reserve(w.n_atoms, 1, 8)
    m.energy_forces(cw, sw, bw, ow)
    with pytest.raises(NNPError) as ei:
        m.status()
    assert ei.value.code == nat.NNP_ECAPACITY
    m.reserve(w.n_atoms, 1, 8)
    r = m.energy_forces(cw, sw, bw, ow, check=True)
    ref = NNPModel(spec, "fp32").energy_forces(cw, sw, bw, ow, check=True)
    torch.cuda.synchronize()
    assert abs(float(r.energy[0]) - float(ref.energy[0])) < 1e-9


def test_autograd_function_gives_minus_forces(m32):
    from paper_2207_14276_amd import NNPFunction
    b = SYSTEMS["ragged16"]
    c, s, bx, o = to_dev(b)
    c = c.clone().requires_grad_(True)
    E = NNPFunction.apply(c, s, bx, o, m32)
    w = torch.linspace(0.5, 1.5, b.n_systems, dtype=torch.float64, device=c.device)
    (E * w).sum().backward()
    r = m32.energy_forces(c.detach(), s, bx, o, check=True)
    g = torch.repeat_interleave(w.float(), torch.as_tensor(np.diff(b.offsets), device=c.device))
    torch.testing.assert_close(c.grad, -g[:, None] * r.forces, rtol=1e-5, atol=1e-6)


def test_autotune_changes_no_result(oracle_lib):
    """Tuning the launch shapes on a batch picks valid shapes and leaves every
    result as it was (tile shapes change no per-element arithmetic)."""
    from paper_2207_14276_amd import NNPModel
    spec = synth.make_model(0)
    b = synth.ragged_solutes(24, seed=31)
    for prec in ("fp32", "bf16"):
        m = NNPModel(spec, prec)
        c, sp, bx, o = to_dev(b)
        r0 = m.energy_forces(c, sp, bx, o, check=True)
        e0, f0 = r0.energy.cpu().numpy(), r0.forces.cpu().numpy()
        tuned = m.autotune(c, sp, bx, o)
        log(f"[autotune {prec}] {tuned}")
        assert tuned, "no site was tuned"
        allowed = lambda k: ((1, 2, 4) if k == "aev_fwd_waves" else (1, 2, 4, 5, 8) if k == "aev_bwd_waves"
                             else (4, 8, 18) if k == "chain_waves" else (64, 128, 256))
        for k, v in tuned.items():
            assert v in allowed(k), (k, v)
        r1 = m.energy_forces(c, sp, bx, o, check=True)
        assert np.array_equal(r1.energy.cpu().numpy(), e0)
        assert float(np.abs(r1.forces.cpu().numpy() - f0).max()) <= 1e-5
        m.close()


def test_calls_only_enqueue(spec):
    """nnp_energy_forces enqueues its work and returns: 64 back-to-back calls
    on the 512-solute batch come back to the host well before the device has
    finished them (a call waits only once 32 earlier calls' descriptor copies
    are still in flight), and every call gives the first call's energies."""
    from paper_2207_14276_amd import NNPModel
    m = NNPModel(spec, "bf16")
    b = synth.config2()
    c, s, bx, o = to_dev(b)
    m.reserve(b.n_atoms, b.n_systems, 160)
    r0 = m.energy_forces(c, s, bx, o, check=True)
    e0 = r0.energy.clone()
    res = [m.energy_forces(c, s, bx, o) for _ in range(4)]  # outputs allocated before timing
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    import time
    start.record()
    t0 = time.perf_counter()
    for k in range(64):
        m.energy_forces(c, s, bx, o, out=res[k % 4])
    t_host = time.perf_counter() - t0
    end.record()
    torch.cuda.synchronize()
    t_dev = start.elapsed_time(end) * 1e-3
    m.status()
    log(f"[enqueue] 64 calls: host {t_host * 1e3:.2f} ms, device {t_dev * 1e3:.2f} ms")
    assert t_host < 0.9 * t_dev
    for r in res:
        assert torch.equal(r.energy, e0)
    m.close()
