"""Pins the oracle's AEV to closed forms of the paper's symmetry functions.

Each expected value here is evaluated with Python's `math` from the formula
as printed (paper, "ANI models": cutoff, radial and angular equations), with
the angle taken from math.acos rather than the oracle's cos/sin split.
"""
import math

import numpy as np
import pytest

import synth

P = synth.aev_params()
D = synth.aev_dim(P)
NS = P["n_species"]
NR = len(P["shf_rad"])
RAD_LEN = NS * NR
BLK = len(P["shf_ang"]) * len(P["shf_z"])


def fc(r, rc):
    return 0.5 * math.cos(math.pi * r / rc) + 0.5 if r <= rc else 0.0


def radial_expected(r, m):
    return 0.25 * math.exp(-P["eta_rad"] * (r - P["shf_rad"][m]) ** 2) * fc(r, P["rc_rad"])


def pair_slot(a, b):
    """Upper-triangle enumeration of unordered species pairs, by counting."""
    k = 0
    for x in range(NS):
        for y in range(x, NS):
            if (x, y) == (min(a, b), max(a, b)):
                return k
            k += 1
    raise AssertionError


def test_aev_dimension_is_1008():
    # 7 radial sub-AEVs of 16 and 28 angular sub-AEVs of 4 x 8 (paper: N radial
    # and N(N+1)/2 angular sub-AEVs for N species)
    assert D == 7 * 16 + 28 * 32 == 1008


@pytest.mark.parametrize("r", [0.95, 1.7, 2.5, 3.3, 4.4, 5.0, 5.0999, 5.1, 5.3, 7.0])
def test_isolated_pair_radial(oracle_lib, r):
    xyz = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]], np.float64)
    # keep the exact float32 distance the oracle will see
    xyz = xyz.astype(np.float32)
    rr = float(xyz[1, 0])
    spec = np.array([synth.H, synth.O], np.int32)
    G = oracle_lib.aev(xyz, spec, np.zeros(3), P)
    for m in range(NR):
        exp_h = radial_expected(rr, m) if rr < P["rc_rad"] else 0.0
        # atom 0 (H) sees an O neighbour, atom 1 (O) sees an H neighbour
        assert G[0, synth.O * NR + m] == pytest.approx(exp_h, rel=1e-13, abs=1e-300)
        assert G[1, synth.H * NR + m] == pytest.approx(exp_h, rel=1e-13, abs=1e-300)
    # nothing else is populated: other radial blocks and all angular terms
    mask = np.ones(D, bool)
    mask[synth.O * NR:(synth.O + 1) * NR] = False
    assert np.all(G[0, mask] == 0.0)


def test_cutoff_function_endpoints():
    # fc(0) = 1, fc(Rc) = 0, fc'(Rc) = 0: a pair at 1e-6 A inside Rc has a
    # radial term that vanishes quadratically
    rc = P["rc_rad"]
    assert fc(0.0, rc) == 1.0
    assert abs(fc(rc, rc)) < 1e-16
    eps = 1e-4
    assert fc(rc - eps, rc) < 1e-7


def _triplet(Rj, Rk, theta, sj, sk):
    xyz = np.array([[0.0, 0.0, 0.0],
                    [Rj, 0.0, 0.0],
                    [Rk * math.cos(theta), Rk * math.sin(theta), 0.0]]).astype(np.float32)
    spec = np.array([synth.C, sj, sk], np.int32)
    return xyz, spec


def angular_expected(xyz, r, a):
    dj = xyz[1].astype(np.float64) - xyz[0]
    dk = xyz[2].astype(np.float64) - xyz[0]
    Rj, Rk = float(np.linalg.norm(dj)), float(np.linalg.norm(dk))
    theta = math.acos(max(-1.0, min(1.0, float(dj @ dk) / (Rj * Rk))))
    f1 = 2.0 ** (1 - P["zeta"]) * (1 + math.cos(theta - P["shf_z"][a])) ** P["zeta"]
    f2 = math.exp(-P["eta_ang"] * ((Rj + Rk) / 2 - P["shf_ang"][r]) ** 2)
    return f1 * f2 * fc(Rj, P["rc_ang"]) * fc(Rk, P["rc_ang"])


@pytest.mark.parametrize("Rj,Rk,theta", [(1.1, 1.4, 1.9), (1.0, 3.0, 0.7), (2.2, 2.2, 2.6),
                                         (1.5, 3.3, 1.2)])
@pytest.mark.parametrize("sj,sk", [(synth.H, synth.H), (synth.H, synth.O), (synth.S, synth.N)])
def test_isolated_triplet_angular(oracle_lib, Rj, Rk, theta, sj, sk):
    xyz, spec = _triplet(Rj, Rk, theta, sj, sk)
    # keep the j-k distance beyond the angular cutoff for centre-0-only terms
    G = oracle_lib.aev(xyz, spec, np.zeros(3), P)
    base = RAD_LEN + BLK * pair_slot(sj, sk)
    for r in range(len(P["shf_ang"])):
        for a in range(len(P["shf_z"])):
            exp = angular_expected(xyz, r, a)
            assert G[0, base + r * len(P["shf_z"]) + a] == pytest.approx(exp, rel=1e-10, abs=1e-300)
    # every other angular block of the centre is empty
    ang = G[0, RAD_LEN:].reshape(-1, BLK)
    others = np.delete(ang, pair_slot(sj, sk), axis=0)
    assert np.all(others == 0.0)


def test_angle_at_shift_gives_prefactor_two(oracle_lib):
    # theta == theta_s,a -> (1 + cos 0)^zeta * 2^(1 - zeta) = 2 exactly
    a = 3
    theta = float(P["shf_z"][a])
    xyz, spec = _triplet(1.3, 1.3, theta, synth.H, synth.H)
    G = oracle_lib.aev(xyz, spec, np.zeros(3), P)
    dj = xyz[1].astype(np.float64)
    dk = xyz[2].astype(np.float64)
    Rj, Rk = np.linalg.norm(dj), np.linalg.norm(dk)
    th = math.acos(float(dj @ dk) / (Rj * Rk))
    base = RAD_LEN + BLK * pair_slot(synth.H, synth.H)
    for r in range(4):
        f2 = math.exp(-P["eta_ang"] * ((Rj + Rk) / 2 - P["shf_ang"][r]) ** 2)
        f1 = 2.0 ** (1 - P["zeta"]) * (1 + math.cos(th - theta)) ** P["zeta"]
        assert f1 == pytest.approx(2.0, rel=1e-12)
        exp = 2.0 * f2 * fc(Rj, P["rc_ang"]) * fc(Rk, P["rc_ang"])
        assert G[0, base + r * 8 + a] == pytest.approx(exp, rel=1e-10)


def test_pair_order_is_unordered(oracle_lib):
    # swapping the species of j and k lands in the same block with the same values
    xyz, spec = _triplet(1.2, 1.6, 1.8, synth.N, synth.O)
    G1 = oracle_lib.aev(xyz, spec, np.zeros(3), P)
    spec2 = spec.copy()
    spec2[1], spec2[2] = spec[2], spec[1]
    xyz2 = xyz.copy()
    xyz2[1], xyz2[2] = xyz[2], xyz[1]
    G2 = oracle_lib.aev(xyz2, spec2, np.zeros(3), P)
    np.testing.assert_allclose(G1[0, RAD_LEN:], G2[0, RAD_LEN:], rtol=1e-13)


def test_symmetric_triangle_blocks(oracle_lib):
    # isosceles triangle centred on atom 0, mirror-symmetric in float32 too:
    # atoms 1 and 2 see mirror-image environments
    c, s_ = 1.4 * math.cos(0.95), 1.4 * math.sin(0.95)
    xyz = np.array([[0, 0, 0], [c, s_, 0], [c, -s_, 0]], np.float32)
    spec = np.array([synth.C, synth.H, synth.H], np.int32)
    G = oracle_lib.aev(xyz, spec, np.zeros(3), P)
    np.testing.assert_allclose(G[1], G[2], rtol=1e-12, atol=1e-300)


def test_triplet_outside_angular_cutoff_has_no_angular_terms(oracle_lib):
    xyz, spec = _triplet(1.2, 3.6, 1.0, synth.H, synth.H)  # Rk beyond 3.5 A
    G = oracle_lib.aev(xyz, spec, np.zeros(3), P)
    assert np.all(G[0, RAD_LEN:] == 0.0)
    assert G[0, synth.H * NR:(synth.H + 1) * NR].sum() > 0.0
