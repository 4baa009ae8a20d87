"""Pins the oracle's analytic forces and virial to finite differences of its
own energy, and the sampled (local) mode to the whole-system mode.

Central differences use h = 1e-5 A.  The cosine cutoff is continuous with a
continuous slope but a jump in curvature at R_c, so a step that straddles a
neighbour's cutoff crossing loses the O(h^2) error; at h = 1e-4 A one atom of
the small periodic box does (error 1e-6, against 7e-10 at h = 3e-5 A).  In
float64 the rounding error at h = 1e-5 A is ~1e-10."""
import numpy as np
import pytest

import synth


def fd_force(oracle_lib, om, s, i, a, h=1e-5):
    x = s.coords.astype(np.float64)
    out = []
    for sgn in (+1, -1):
        y = x.copy()
        y[i, a] += sgn * h
        E, _, _, _ = _energy64(oracle_lib, om, y, s.species, s.box)
        out.append(E)
    return -(out[0] - out[1]) / (2 * h)


def _energy64(oracle_lib, om, x64, species, box):
    """Energy at float64 coordinates (bypasses the float32 input rounding)."""
    import ctypes as C
    lib = oracle_lib._load()
    x = np.ascontiguousarray(x64, dtype=np.float64)
    s = np.ascontiguousarray(species, dtype=np.int32)
    b = np.ascontiguousarray(np.asarray(box, np.float32).astype(np.float64))
    e_atom = np.zeros(len(s))
    E = np.zeros(1)
    rc = lib.orc_energy_forces(len(s), oracle_lib._dp(x), oracle_lib._ip(s), oracle_lib._dp(b),
                               C.byref(om.struct), oracle_lib._dp(e_atom), oracle_lib._dp(E),
                               None, None)
    assert rc == 0
    return float(E[0]), e_atom, None, None


def _check_fd(oracle_lib, om, s, atoms, tol_rel=1e-6):
    _, _, F, _ = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    scale = np.abs(F).max()
    for i in atoms:
        for a in range(3):
            fd = fd_force(oracle_lib, om, s, int(i), a)
            assert abs(fd - F[i, a]) <= tol_rel * scale + 1e-10, (i, a, fd, F[i, a])


def test_fd_small_cluster(oracle_lib):
    s = synth.config0()
    om = oracle_lib.OracleModel(synth.make_model(0))
    _check_fd(oracle_lib, om, s, range(s.n))


def test_fd_small_periodic_box_with_self_images(oracle_lib):
    s = synth.water_box(8, seed=5)   # L ~ 6.2 A: several images of each atom
    om = oracle_lib.OracleModel(synth.make_model(1))
    _check_fd(oracle_lib, om, s, range(s.n))


def test_fd_dense_solute_two_network_ensemble(oracle_lib):
    s = synth.ragged_solutes(1, seed=9, nmin=60, nmax=60).systems[0]
    om = oracle_lib.OracleModel(synth.make_model(2, n_ensemble=2))
    _check_fd(oracle_lib, om, s, range(0, s.n, 7))


def test_fd_water_box_16_atoms(oracle_lib):
    s = synth.config1()
    om = oracle_lib.OracleModel(synth.make_model(0))
    rng = np.random.default_rng(1)
    atoms = rng.choice(s.n, 16, replace=False)
    # one random component per atom keeps the CPU suite short
    _, _, F, _ = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    scale = np.abs(F).max()
    for i in atoms:
        a = int(rng.integers(0, 3))
        fd = fd_force(oracle_lib, om, s, int(i), a)
        assert abs(fd - F[i, a]) <= 1e-6 * scale + 1e-10


def test_virial_matches_strain_derivative(oracle_lib):
    # non-periodic: any strain eps gives dE/deps_ab = -W_ba
    s = synth.config0()
    om = oracle_lib.OracleModel(synth.make_model(3))
    _, _, F, W = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    x = s.coords.astype(np.float64)
    np.testing.assert_allclose(W, x.T @ F, rtol=1e-10, atol=1e-12)
    h = 1e-5
    for a in range(3):
        for b in range(3):
            E = []
            for sgn in (+1, -1):
                eps = np.zeros((3, 3))
                eps[a, b] = sgn * h
                E.append(_energy64(oracle_lib, om, x @ (np.eye(3) + eps).T, s.species, s.box)[0])
            dE = (E[0] - E[1]) / (2 * h)
            assert dE == pytest.approx(-W[b, a], rel=1e-6, abs=1e-9)


def test_virial_periodic_axis_strain(oracle_lib):
    # periodic: scaling one axis (coordinates and box) gives dE/deps_aa = -W_aa
    s = synth.water_box(30, seed=2)
    om = oracle_lib.OracleModel(synth.make_model(4))
    _, _, _, W = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    x = s.coords.astype(np.float64)
    h = 1e-5
    for a in range(3):
        E = []
        for sgn in (+1, -1):
            sc = np.ones(3)
            sc[a] += sgn * h
            # the box is passed as float64 here so the strain is exact
            import ctypes as C
            lib = oracle_lib._load()
            xx = np.ascontiguousarray(x * sc)
            bb = np.ascontiguousarray(s.box.astype(np.float64) * sc)
            sp = np.ascontiguousarray(s.species, np.int32)
            ea = np.zeros(s.n)
            EE = np.zeros(1)
            lib.orc_energy_forces(s.n, oracle_lib._dp(xx), oracle_lib._ip(sp), oracle_lib._dp(bb),
                                  C.byref(om.struct), oracle_lib._dp(ea), oracle_lib._dp(EE),
                                  None, None)
            E.append(EE[0])
        dE = (E[0] - E[1]) / (2 * h)
        assert dE == pytest.approx(-W[a, a], rel=1e-6, abs=1e-9)


def test_sampled_equals_whole_system(oracle_lib):
    om = oracle_lib.OracleModel(synth.make_model(0))
    for s in (synth.config1(), synth.water_box(8, seed=5), synth.config0()):
        _, ea, F, _ = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
        t = np.arange(0, s.n, max(1, s.n // 12))
        e, f = oracle_lib.sampled(s.coords, s.species, s.box, om, t)
        np.testing.assert_allclose(e, ea[t], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(f, F[t], rtol=1e-11, atol=1e-13)


def test_collinear_triplet_force_is_the_central_difference(oracle_lib):
    """At an exactly collinear triplet the sine of the angle, |d_j x d_k| /
    (R_j R_k), has a kink, and the oracle takes its derivative as zero there
    (the reading of the gradient at collinear triplets).  That is exactly the
    central difference of the energy: the one-sided slopes of |sin| across
    the line are opposite and cancel.  The case is not trivial: the one-sided
    slopes across the line differ."""
    om = oracle_lib.OracleModel(synth.make_model(0))
    # C at the origin between an H and an O on the x axis: theta = pi
    x = np.array([[0.0, 0.0, 0.0], [1.25, 0.0, 0.0], [-1.125, 0.0, 0.0]])
    sp = np.array([1, 0, 3], np.int32)
    box = np.zeros(3, np.float32)
    E0, _, F, _ = oracle_lib.energy_forces(x.astype(np.float32), sp, box, om)
    h = 1e-5
    for i in range(3):
        for a in range(3):
            e = []
            for sgn in (+1, -1):
                y = x.copy()
                y[i, a] += sgn * h
                e.append(_energy64(oracle_lib, om, y, sp, box)[0])
            assert F[i, a] == pytest.approx(-(e[0] - e[1]) / (2 * h), abs=1e-7), (i, a)
    # across the line (the centre moved along y) the one-sided slopes differ
    up, down = x.copy(), x.copy()
    up[0, 1] += h
    down[0, 1] -= h
    s_up = (_energy64(oracle_lib, om, up, sp, box)[0] - E0) / h
    s_down = (E0 - _energy64(oracle_lib, om, down, sp, box)[0]) / h
    assert abs(s_up - s_down) > 1e-4
