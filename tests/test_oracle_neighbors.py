"""Pins the oracle's brute-force periodic neighbour search.

The counts for a simple cubic lattice are the textbook coordination shells
(6, 12, 8, 6, 24, 24 lattice vectors with |n|^2 = 1..6), independent of how
many atoms the periodic box holds: each periodic image inside the cutoff is a
distinct neighbour, self-images included.
"""
import numpy as np
import pytest

import synth

SHELLS = {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24}


def lattice(n_side, a):
    g = np.arange(n_side) * a + 0.1
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)


def expected_count(rc, a):
    return sum(c for k, c in SHELLS.items() if k * a * a < rc * rc)


@pytest.mark.parametrize("n_side", [1, 2, 4])
@pytest.mark.parametrize("rc", [2.5, 3.0, 3.5, 4.1, 4.5, 5.1])
def test_simple_cubic_counts(oracle_lib, n_side, rc):
    a = 2.0
    xyz = lattice(n_side, a)
    box = np.full(3, n_side * a, np.float32)
    for i in (0, len(xyz) - 1):
        nb = oracle_lib.neighbours(xyz, box, rc, i)
        assert len(nb) == expected_count(rc, a)
        assert len(set(nb)) == len(nb)  # each (j, image) once


def test_nonperiodic_has_no_images(oracle_lib):
    xyz = lattice(3, 2.0)
    nb = oracle_lib.neighbours(xyz, np.zeros(3), 2.5, 13)  # centre of the 3x3x3 cube
    assert len(nb) == 6
    assert all(img == (0, 0, 0) for _, img in nb)


def test_image_shift_invariance(oracle_lib):
    # moving atoms by whole box vectors changes nothing (coordinates need not be wrapped)
    w = synth.water_box(20, seed=7)
    p = synth.aev_params()
    G0 = oracle_lib.aev(w.coords, w.species, w.box, p)
    rng = np.random.default_rng(0)
    shifted = w.coords.astype(np.float64) + rng.integers(-2, 3, size=w.coords.shape) * w.box
    G1 = oracle_lib.aev(shifted.astype(np.float32), w.species, w.box, p)
    # float32 rounding of the shifted coordinates perturbs positions by ~1e-6 A
    np.testing.assert_allclose(G0, G1, atol=2e-4)


def test_small_box_needs_several_images(oracle_lib):
    # 20 waters: L ~ 5.85 A < 2 * 5.1 A, so an atom sees several images of itself
    w = synth.water_box(7, seed=3)
    assert w.box[0] < 2 * 5.1
    nb = oracle_lib.neighbours(w.coords, w.box, 5.1, 0)
    selfs = [img for j, img in nb if j == 0]
    assert len(selfs) == expected_count(5.1, float(w.box[0]))
