"""Pins the oracle with invariances the energy must have: translation,
rotation, same-species permutation, periodic wrapping; zero net force and
torque; continuity of energy and force when a neighbour crosses a cutoff."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def om(oracle_lib):
    return oracle_lib.OracleModel(synth.make_model(0))


def _rot(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _e64(oracle_lib, om, x, species, box):
    from tests.test_oracle_fd import _energy64
    return _energy64(oracle_lib, om, x, species, box)


def test_translation_rotation(oracle_lib, om):
    s = synth.config0()
    x = s.coords.astype(np.float64)
    E0, ea0, _, _ = _e64(oracle_lib, om, x, s.species, s.box)
    E1, ea1, _, _ = _e64(oracle_lib, om, x + np.array([3.3, -7.1, 0.4]), s.species, s.box)
    R = _rot(4)
    E2, ea2, _, _ = _e64(oracle_lib, om, (x - x.mean(0)) @ R.T, s.species, s.box)
    assert E1 == pytest.approx(E0, rel=1e-12)
    assert E2 == pytest.approx(E0, rel=1e-12)
    np.testing.assert_allclose(ea2, ea0, rtol=1e-10, atol=1e-13)


def test_same_species_permutation(oracle_lib, om):
    s = synth.config0()
    perm = np.arange(s.n)
    for sp in range(4):
        idx = np.where(s.species == sp)[0]
        perm[idx] = idx[::-1]
    E0, ea0, F0, _ = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    E1, ea1, F1, _ = oracle_lib.energy_forces(s.coords[perm], s.species[perm], s.box, om)
    assert E1 == pytest.approx(E0, rel=1e-12)
    np.testing.assert_allclose(ea1, ea0[perm], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(F1, F0[perm], rtol=1e-10, atol=1e-13)


def test_net_force_and_torque_vanish(oracle_lib, om):
    s = synth.config0()
    _, _, F, _ = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    x = s.coords.astype(np.float64)
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-12 * scale * s.n
    assert np.abs(np.cross(x, F).sum(0)).max() < 1e-11 * scale * s.n
    w = synth.config1()
    _, _, Fw, _ = oracle_lib.energy_forces(w.coords, w.species, w.box, om)
    assert np.abs(Fw.sum(0)).max() < 1e-11 * np.abs(Fw).max() * np.sqrt(w.n)


@pytest.mark.parametrize("rc_name,species", [("rc_rad", (synth.C, synth.N)),
                                             ("rc_ang", (synth.H, synth.O))])
def test_continuity_across_cutoff(oracle_lib, om, rc_name, species):
    """A neighbour crossing a cutoff leaves energy and force continuous: the
    cutoff and its slope vanish at R_c.  The second difference
    E(rc+d) - 2E(rc) + E(rc-d) is then O(d^2) (a value jump would make it O(1),
    a kink O(d)) and the force difference across rc is O(d)."""
    import ctypes as C
    lib = oracle_lib._load()
    rc = om.spec.aev[rc_name]
    sp = np.array([species[0], species[1], species[1]], np.int32)

    def ef(r):
        # centre at the origin, one fixed close neighbour, one at distance r
        x = np.ascontiguousarray(np.array([[0.0, 0, 0], [1.1, 0.0, 0.0], [0.0, r, 0.0]]))
        F = np.zeros((3, 3))
        ea = np.zeros(3)
        EE = np.zeros(1)
        lib.orc_energy_forces(3, oracle_lib._dp(x), oracle_lib._ip(sp),
                              oracle_lib._dp(np.zeros(3)), C.byref(om.struct),
                              oracle_lib._dp(ea), oracle_lib._dp(EE), oracle_lib._dp(F), None)
        return EE[0], F

    E0, _ = ef(rc)
    sd, fj = [], []
    for delta in (1e-2, 1e-3, 1e-4):
        Ep, Fp = ef(rc + delta)
        Em, Fm = ef(rc - delta)
        sd.append(abs(Ep - 2 * E0 + Em))
        fj.append(np.abs(Fp - Fm).max())
    assert sd[1] < sd[0] / 30 + 1e-15
    assert sd[2] < sd[1] / 30 + 1e-15
    assert fj[1] < fj[0] / 5 + 1e-13
    assert fj[2] < fj[1] / 5 + 1e-13
