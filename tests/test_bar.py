"""The library's Bennett acceptance ratio estimator (nnp_bar, host code)
against closed forms: a constant energy shift (exact), harmonic states
whose free-energy difference is (1/2) ln(k_1/k_0) per dimension, unequal
sample sizes, reweighting from a reference ensemble to a target one,
antisymmetry under exchange of the states, and the error paths."""
import numpy as np
import pytest

from paper_2207_14276_amd import NNPError
from paper_2207_14276_amd.bar import bar, bar_reduced, bar_reweighted, beta_at


def harmonic_samples(rng, k, n, dim=3):
    # x ~ exp(-k x^2 / 2) at beta = 1
    return rng.normal(0.0, 1.0 / np.sqrt(k), size=(n, dim))


def energy(x, k):
    return 0.5 * k * (x * x).sum(1)


def test_constant_shift_is_exact():
    rng = np.random.default_rng(0)
    for d in (-3.0, 0.0, 0.7, 12.5):
        U0_0 = rng.normal(size=400)
        U0_1 = rng.normal(size=300)
        est, _ = bar(U0_0, U0_0 + d, U0_1, U0_1 + d, beta=1.0)
        assert est == pytest.approx(d, abs=1e-9)


@pytest.mark.parametrize("n0,n1", [(40000, 40000), (10000, 40000), (40000, 8000)])
def test_harmonic_states(n0, n1):
    rng = np.random.default_rng(1)
    k0, k1, dim = 1.0, 2.5, 3
    x0, x1 = harmonic_samples(rng, k0, n0, dim), harmonic_samples(rng, k1, n1, dim)
    est, sig = bar(energy(x0, k0), energy(x0, k1), energy(x1, k0), energy(x1, k1), beta=1.0)
    exact = 0.5 * dim * np.log(k1 / k0)
    assert 0.0 < sig < 0.02
    assert abs(est - exact) < 4.0 * sig


def test_kcal_units_and_temperature():
    """beta scales consistently: states at 300 K with energies in kcal/mol."""
    rng = np.random.default_rng(2)
    beta = beta_at(300.0)
    k0, k1 = 1.0 / beta, 3.0 / beta      # force constants in kcal/mol per unit^2
    x0 = rng.normal(0.0, 1.0 / np.sqrt(beta * k0), size=(30000, 2))
    x1 = rng.normal(0.0, 1.0 / np.sqrt(beta * k1), size=(30000, 2))
    est, sig = bar(energy(x0, k0), energy(x0, k1), energy(x1, k0), energy(x1, k1), beta)
    exact = (1.0 / beta) * 0.5 * 2 * np.log(k1 / k0)
    assert abs(est - exact) < 4.0 * sig


def test_reweighting_to_a_target_ensemble():
    """Samples of reference harmonic states (k0, k1) reweighted to target
    harmonic states (k0', k1') give the target's (1/2) ln(k1'/k0')."""
    rng = np.random.default_rng(3)
    k0, k1, t0, t1, dim, n = 1.0, 2.0, 1.2, 2.3, 2, 60000
    x0, x1 = harmonic_samples(rng, k0, n, dim), harmonic_samples(rng, k1, n, dim)
    est, sig = bar_reweighted(energy(x0, k0), energy(x0, k1), energy(x1, k0), energy(x1, k1),
                              energy(x0, t0), energy(x0, t1), energy(x1, t0), energy(x1, t1), beta=1.0)
    exact = 0.5 * dim * np.log(t1 / t0)
    assert 0.0 < sig < 0.05
    assert abs(est - exact) < 4.0 * sig
    # and differs from the reference ensemble's own difference
    ref = 0.5 * dim * np.log(k1 / k0)
    assert abs(est - ref) > 10.0 * sig


def test_zero_log_weights_equal_unweighted():
    rng = np.random.default_rng(4)
    u, v = rng.normal(1.0, 0.5, 500), rng.normal(-0.8, 0.6, 700)
    a = bar_reduced(u, v)
    b = bar_reduced(u, v, np.zeros(500), np.zeros(700))
    assert a[0] == pytest.approx(b[0], abs=1e-12)
    assert a[1] == pytest.approx(b[1], rel=1e-9)


def test_exchanging_the_states_negates():
    rng = np.random.default_rng(5)
    u, v = rng.normal(2.0, 1.0, 900), rng.normal(-1.5, 1.2, 600)
    d, s = bar_reduced(u, v)
    d2, s2 = bar_reduced(v, u)
    assert d2 == pytest.approx(-d, abs=1e-9)
    assert s2 == pytest.approx(s, rel=1e-6)


def test_errors():
    with pytest.raises(NNPError):
        bar_reduced(np.zeros(0), np.zeros(3))
    with pytest.raises(NNPError):
        bar_reduced(np.array([1.0, np.nan]), np.zeros(3))
    with pytest.raises(ValueError):
        bar_reduced(np.zeros(3), np.zeros(3), np.zeros(2), None)
