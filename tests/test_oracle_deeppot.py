"""Pins the oracle's DeepPot-style descriptor (section "DeePMD Models") and
its analytic gradient to closed forms, invariances and finite differences.

Closed forms: a lone pair gives {1/R, 1, 0, 0} in the neighbour's species
block; a bent triatomic gives {1/R, cos t, sin t, 0} for the second
neighbour whatever the orientation, and a third neighbour's (x, y, z) are its
coordinates in the right-handed frame of the first two; a single atom in a
5 A periodic box sees its six images at exactly equal distance, which fixes
the tie order (neighbour index, then image x, y, z ascending) and the frame
signs; with small per-species capacities the farthest neighbours of a
species are dropped and the frame still uses the two nearest overall.

The descriptor has no smoothing at the cutoff and changes slot order when two
neighbours of a species swap distance order, so the energy is only
piecewise smooth; the finite-difference systems are checked first to sit at
least 3e-5 A away from every such boundary (h = 1e-5 A)."""
import numpy as np
import pytest

import synth
from tests.test_oracle_fd import _energy64

P = synth.dp_params()
SEL = np.array(P["sel"])
OFF = np.concatenate([[0], np.cumsum(SEL)])   # first slot of each species block


def desc(oracle_lib, x, sp, box=None, p=P):
    box = np.zeros(3) if box is None else box
    return oracle_lib.dp_descriptor(np.asarray(x, np.float32), np.asarray(sp, np.int32), box, p)


def rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_lone_pair(oracle_lib):
    for R in (0.8, 2.5, 5.99):
        x = np.array([[0.0, 0.0, 0.0], [0.0, R, 0.0]], np.float32)
        G = desc(oracle_lib, x, [synth.C, synth.O])
        R32 = float(np.float32(R))
        want = np.zeros((2, 480))
        want[0, 4 * OFF[synth.O]:4 * OFF[synth.O] + 4] = [1 / R32, 1, 0, 0]
        want[1, 4 * OFF[synth.C]:4 * OFF[synth.C] + 4] = [1 / R32, 1, 0, 0]
        np.testing.assert_allclose(G, want, rtol=1e-15, atol=1e-15)
    x = np.array([[0.0, 0.0, 0.0], [6.01, 0.0, 0.0]], np.float32)
    assert np.all(desc(oracle_lib, x, [synth.C, synth.O]) == 0.0)


def test_triatomic_and_out_of_plane_neighbour(oracle_lib):
    rng = np.random.default_rng(0)
    t = 1.83
    p3 = np.array([-1.1, 0.7, -1.6])           # a carbon below the plane
    for _ in range(5):
        Q = rotation(rng)
        local = np.array([[0, 0, 0], [0.95, 0, 0], [0.97 * np.cos(t), 0.97 * np.sin(t), 0], p3])
        x = (local @ Q.T + rng.normal(size=3) * 3).astype(np.float32)
        G = desc(oracle_lib, x, [synth.O, synth.H, synth.H, synth.C])[0]
        np.testing.assert_allclose(G[0:4], [1 / 0.95, 1, 0, 0], atol=2e-6)
        np.testing.assert_allclose(G[4:8], [1 / 0.97, np.cos(t), np.sin(t), 0], atol=2e-6)
        r3 = np.linalg.norm(p3)
        c = 4 * OFF[synth.C]
        np.testing.assert_allclose(G[c:c + 4], [1 / r3, *(p3 / r3)], atol=2e-6)
        rest = np.ones(480, bool)
        rest[0:8] = rest[c:c + 4] = False
        assert np.all(G[rest] == 0.0)


def test_single_atom_small_box_ties(oracle_lib):
    """Six images at 5 A, all at the same float64 distance: ordered by image
    (-x, -y, -z, +z, +y, +x); e_x = -x, e_y = -y, e_z = e_x x e_y = +z."""
    x = np.array([[1.25, 2.5, 0.75]], np.float32)
    G = desc(oracle_lib, x, [synth.H], box=np.full(3, 5.0, np.float32))[0]
    want = np.zeros(480)
    rows = [[0.2, 1, 0, 0], [0.2, 0, 1, 0], [0.2, 0, 0, -1], [0.2, 0, 0, 1],
            [0.2, 0, -1, 0], [0.2, -1, 0, 0]]
    want[:24] = np.ravel(rows)
    np.testing.assert_array_equal(G, want)


def test_species_blocks_order_and_capacity(oracle_lib):
    """sel = 2 H, 1 of each other species: H at 1.0 and 1.5 kept in that
    order, H at 2.0 and 2.5 dropped; of two O only the nearer one is kept;
    the frame is (H at 1.0, O at 1.2) across species."""
    p = synth.dp_params(sel=(2, 1, 1, 1, 1, 1, 1))
    u = [np.array(v, float) / np.linalg.norm(v) for v in
         ([1, 0, 0], [0.3, 1, 0], [0, 0.4, 1], [-1, 0.2, 0.1], [0.5, -1, 0.3], [0.2, 0.2, -1])]
    pos = [np.zeros(3), 1.0 * u[0], 1.5 * u[1], 2.0 * u[2], 2.5 * u[3], 1.2 * u[4], 3.0 * u[5]]
    sp = [synth.C, synth.H, synth.H, synth.H, synth.H, synth.O, synth.O]
    x = np.array(pos, np.float32)
    G = desc(oracle_lib, x, sp, p=p)[0]
    d = x.astype(np.float64) - x[0]
    ex = d[1] / np.linalg.norm(d[1])
    uo = d[5] - (d[5] @ ex) * ex
    ey = uo / np.linalg.norm(uo)
    ez = np.cross(ex, ey)
    F = np.stack([ex, ey, ez])

    def feat(k):
        R = np.linalg.norm(d[k])
        return np.concatenate([[1 / R], F @ d[k] / R])

    want = np.zeros(4 * 8)
    want[0:4], want[4:8] = feat(1), feat(2)       # H block: slots 0, 1
    o = 4 * (2 + 1 + 1)                           # O block after H(2), C(1), N(1)
    want[o:o + 4] = feat(5)
    np.testing.assert_allclose(G, want, rtol=1e-12, atol=1e-14)


def test_rotation_translation_permutation(oracle_lib):
    rng = np.random.default_rng(3)
    s = synth.random_solute(rng, 40, 1.2 * 40 ** (1 / 3), synth.CONFIG2_PROBS)
    G = desc(oracle_lib, s.coords, s.species)
    Q = rotation(rng)
    x2 = (s.coords.astype(np.float64) @ Q.T + [4.0, -2.0, 7.0]).astype(np.float32)
    np.testing.assert_allclose(desc(oracle_lib, x2, s.species), G, atol=2e-5)
    perm = rng.permutation(s.n)
    Gp = desc(oracle_lib, s.coords[perm], s.species[perm])
    np.testing.assert_array_equal(Gp, G[perm])


def test_periodic_equals_supercell(oracle_lib):
    """Box of 13 A (> 2 rc): each atom's periodic descriptor equals that of
    the central copy in an explicit 3 x 3 x 3 non-periodic supercell."""
    rng = np.random.default_rng(4)
    L = np.float32(13.0)
    s = synth.random_solute(rng, 120, 13.0, synth.CONFIG2_PROBS)
    x = np.mod(s.coords, L).astype(np.float32)
    G = desc(oracle_lib, x, s.species, box=np.full(3, L, np.float32))
    shifts = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    sc = np.concatenate([x.astype(np.float64) + np.array(t) * float(L) for t in shifts]).astype(np.float32)
    centre = shifts.index((0, 0, 0))
    Gs = desc(oracle_lib, sc, np.tile(s.species, len(shifts)))[centre * s.n:(centre + 1) * s.n]
    np.testing.assert_allclose(Gs, G, atol=2e-6)
    assert np.count_nonzero(G) > 0


def boundary_gap(x, species, box, p=P):
    """Smallest distance of the system to a descriptor discontinuity: |R - rc|
    over all neighbours; within each species, the gaps between consecutive
    kept distances and between the last kept one and the first dropped one;
    and the gaps among the three nearest neighbours (the frame's pair)."""
    rc, sel = p["rc"], p["sel"]
    x = np.asarray(x, np.float64)
    L = np.asarray(box, np.float64)
    per = L > 0
    k = [int(np.ceil(rc / L[a])) + 1 if per[a] else 0 for a in range(3)]
    sh = np.array([(a, b, c) for a in range(-k[0], k[0] + 1) for b in range(-k[1], k[1] + 1)
                   for c in range(-k[2], k[2] + 1)], float) * np.where(per, L, 0.0)
    sp_all = np.tile(np.asarray(species), len(sh))
    gap = np.inf
    for i in range(len(x)):
        r = np.linalg.norm(x[None, :, :] + sh[:, None, :] - x[i], axis=-1).ravel()
        keep = (r > 0) & (r < rc + 0.5)
        r, sp = r[keep], sp_all[keep]
        if len(r):
            gap = min(gap, np.abs(r - rc).min())
        inside = r < rc
        r, sp = r[inside], sp[inside]
        gap = min(gap, np.diff(np.sort(r)[:3]).min(initial=np.inf))
        for s_ in range(len(sel)):
            rs = np.sort(r[sp == s_])[:sel[s_] + 1]
            if len(rs) > 1:
                gap = min(gap, np.diff(rs).min())
    return gap


def _check_fd(oracle_lib, om, s, atoms, tol_rel=1e-6, h=1e-5):
    assert boundary_gap(s.coords, s.species, s.box, om.spec.aev) > 3 * h
    _, _, F, _ = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
    scale = np.abs(F).max()
    x = s.coords.astype(np.float64)
    for i in atoms:
        for a in range(3):
            e = []
            for sgn in (+1, -1):
                y = x.copy()
                y[i, a] += sgn * h
                e.append(_energy64(oracle_lib, om, y, s.species, s.box)[0])
            fd = -(e[0] - e[1]) / (2 * h)
            assert abs(fd - F[i, a]) <= tol_rel * scale + 1e-10, (i, a, fd, F[i, a])


@pytest.fixture(scope="module")
def dp_om(oracle_lib):
    return oracle_lib.OracleModel(synth.make_dp_model(0))


def test_fd_cluster(oracle_lib, dp_om):
    s = synth.config0()
    _check_fd(oracle_lib, dp_om, s, range(s.n))


def test_fd_periodic_water(oracle_lib, dp_om):
    s = synth.water_box(12, seed=7)   # L ~ 7.1 A: images of every atom inside rc
    _check_fd(oracle_lib, dp_om, s, range(0, s.n, 2))


def test_fd_capacity_limited(oracle_lib):
    """Small capacities drop neighbours: the dropped ones get no force."""
    om = oracle_lib.OracleModel(synth.make_dp_model(2, dp=synth.dp_params(sel=(3, 2, 1, 2, 1, 1, 1))))
    s = synth.config0()
    _check_fd(oracle_lib, om, s, range(0, s.n, 3))


def test_virial_forces_and_sampled(oracle_lib, dp_om):
    s = synth.config0()
    E, ea, F, W = oracle_lib.energy_forces(s.coords, s.species, s.box, dp_om)
    assert E == pytest.approx(ea.sum(), rel=1e-14)
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-10 * np.abs(F).max())
    rF = s.coords.astype(np.float64).T @ F
    np.testing.assert_allclose(W, rF, atol=1e-9 * np.abs(W).max())
    t = np.arange(0, s.n, 4)
    e_t, f_t = oracle_lib.sampled(s.coords, s.species, s.box, dp_om, t)
    np.testing.assert_allclose(e_t, ea[t], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(f_t, F[t], rtol=1e-10, atol=1e-12)
    w = synth.water_box(12, seed=7)
    _, ea, F, _ = oracle_lib.energy_forces(w.coords, w.species, w.box, dp_om)
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-10 * np.abs(F).max())
    e_t, f_t = oracle_lib.sampled(w.coords, w.species, w.box, dp_om, [0, 5, 17])
    np.testing.assert_allclose(f_t, F[[0, 5, 17]], rtol=1e-10, atol=1e-12)
