"""Pins the oracle's element networks to library routines.

The per-atom energy is recomputed from the oracle's AEV with torch float64
(torch.nn.functional.linear and torch's CELU, the textbook dense routines),
and dE/dG with torch autograd.  The ensemble is pinned as the mean of its
members and the batch as the concatenation of its systems.
"""
import numpy as np
import pytest
import torch

import synth


def _celu_expm1(h, alpha):
    # CELU by its definition on torch primitives; torch's own CPU CELU
    # backward is only ~1e-8 accurate, so autograd differentiates this one
    return torch.where(h > 0, h, alpha * torch.expm1(h / alpha))


def torch_energy(spec, member, species, G, celu=None):
    """Energy of one network with torch float64 library layers."""
    h = torch.as_tensor(G, dtype=torch.float64)
    w = spec.widths[species]
    for m, s, l, ws, bs, n_out, n_in in spec.layer_slices():
        if m != member or s != species:
            continue
        W = torch.as_tensor(spec.weights[ws].astype(np.float64)).reshape(n_out, n_in)
        b = torch.as_tensor(spec.weights[bs].astype(np.float64))
        h = torch.nn.functional.linear(h, W, b)
        if l < len(w) - 2:
            h = (celu or torch.nn.functional.celu)(h, alpha=spec.celu_alpha)
    return h.squeeze(-1)


@pytest.fixture(scope="module")
def small():
    return synth.config0()


def test_atom_energy_matches_torch(oracle_lib, small):
    spec = synth.make_model(11)
    om = oracle_lib.OracleModel(spec)
    G = oracle_lib.aev(small.coords, small.species, small.box, spec.aev)
    _, e_atom, _, _ = oracle_lib.energy_forces(small.coords, small.species, small.box, om)
    for i in range(small.n):
        ref = torch_energy(spec, 0, int(small.species[i]), G[i]).item()
        assert e_atom[i] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_net_gradient_matches_autograd(oracle_lib, small):
    spec = synth.make_model(12)
    om = oracle_lib.OracleModel(spec)
    G = oracle_lib.aev(small.coords, small.species, small.box, spec.aev)
    for s in range(7):
        g = torch.tensor(G[s % small.n], dtype=torch.float64, requires_grad=True)
        E = torch_energy(spec, 0, s, g, celu=_celu_expm1)
        E.backward()
        E_o, dG = oracle_lib.net_energy(om, 0, s, G[s % small.n])
        assert E_o == pytest.approx(E.item(), rel=1e-12)
        np.testing.assert_allclose(dG, g.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_ensemble_is_mean_of_members(oracle_lib, small):
    ens = synth.make_model(5, n_ensemble=3)
    om = oracle_lib.OracleModel(ens)
    E, ea, F, W = oracle_lib.energy_forces(small.coords, small.species, small.box, om)
    # each member alone: the same seed stream gives the same weights
    Es, Fs = [], []
    for m in range(3):
        one = synth.ModelSpec(ens.aev, 1, ens.widths, _member_weights(ens, m), ens.celu_alpha)
        e1, _, f1, _ = oracle_lib.energy_forces(small.coords, small.species, small.box,
                                                oracle_lib.OracleModel(one))
        Es.append(e1)
        Fs.append(f1)
    assert E == pytest.approx(np.mean(Es), rel=1e-13)
    np.testing.assert_allclose(F, np.mean(Fs, axis=0), rtol=1e-11, atol=1e-14)


def _member_weights(spec, member):
    per = spec.weights.size // spec.n_ensemble
    return spec.weights[member * per:(member + 1) * per].copy()


def test_batch_is_concatenation(oracle_lib):
    b = synth.ragged_solutes(4, seed=21, nmin=10, nmax=30)
    om = oracle_lib.OracleModel(synth.make_model(0))
    res = oracle_lib.batch_energy_forces(b, om)
    for k in range(b.n_systems):
        s = b.systems[k]
        E, ea, F, W = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
        assert res["energy"][k] == E
        np.testing.assert_array_equal(res["forces"][k], F)
