"""Dense solutes at the large end of the serving trace's size range, on the
GPU through the C ABI, against the whole-system FP64 oracle.

The serving workload draws request sizes log-uniformly between 20 and 5,000
atoms, half of them non-periodic solutes built like the ragged batch (RSA in
a cube of side 1.2 A n^(1/3), 0.579 atoms per cubic Angstrom).  At 5,000
atoms a centre has ~320 radial neighbours inside 5.1 A and ~100 angular ones
inside 3.5 A (~5k neighbour pairs), so these systems run at the neighbour
capacity of 640 that the server uses.  Every atom's energy and force is
compared, in float32 and with bfloat16 dense layers, once through
nnp_energy_forces and once as the last step of a served request; no
capacity flag may be raised.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import BF16_E_PER_ATOM, BF16_F, FP32_E_ATOM, FP32_F, log, run_gpu, virial_bound

pytestmark = pytest.mark.gpu

SIZES = (2000, 5000)
CAP = 640


def _solute(n):
    return synth.random_solute(np.random.default_rng(40 + n), n, 1.2 * n ** (1.0 / 3.0), synth.CONFIG2_PROBS)


@pytest.fixture(scope="module")
def spec():
    return synth.make_model(0)


@pytest.fixture(scope="module")
def om(oracle_lib, spec):
    return oracle_lib.OracleModel(spec)


@pytest.fixture(scope="module")
def solutes():
    return {n: _solute(n) for n in SIZES}


@pytest.fixture(scope="module")
def refs(oracle_lib, om, solutes):
    out = {}
    for n, s in solutes.items():
        x = s.coords.astype(np.float64)
        d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
        np.fill_diagonal(d, np.inf)
        nr, na = int((d < 5.1).sum(1).max()), int((d < 3.5).sum(1).max())
        E, ea, F, W = oracle_lib.energy_forces(s.coords, s.species, s.box, om)
        log(f"[large n={n}] max radial neighbours {nr}, max angular {na} "
            f"({na * (na - 1) // 2} pairs), oracle E={E:.4f}")
        out[n] = dict(E=E, ea=ea, F=F, W=W, max_rad=nr, max_ang=na)
    return out


def _compare(label, n, e, ea, f, w, ref, coords, e_tol_atom, e_tol_sys, f_tol):
    de_sys = abs(e - ref["E"]) / n
    df = float(np.abs(f - ref["F"]).max())
    msg = f"[{label} n={n}] |dE_s|/N={de_sys:.3e} max|dF|={df:.3e}"
    if ea is not None:
        de_atom = float(np.abs(ea - ref["ea"]).max())
        msg += f" max|dE_i|={de_atom:.3e}"
        if e_tol_atom is not None:
            assert de_atom <= e_tol_atom
    if w is not None:
        dw = float(np.abs(w - ref["W"]).max())
        bound = virial_bound(coords, None, f, ref["F"], w_ref=ref["W"])
        msg += f" max|dW|={dw:.3e} (bound {bound:.3e})"
        assert dw <= bound
    log(msg)
    assert de_sys <= e_tol_sys
    assert df <= f_tol


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_dense_solutes_match_oracle(spec, solutes, refs, prec):
    from paper_2207_14276_amd import NNPModel
    m = NNPModel(spec, prec)
    b = synth.make_batch([solutes[n] for n in SIZES])
    m.reserve(b.n_atoms, b.n_systems, CAP)
    g = run_gpu(m, b, check=False)
    mx = m.status()   # raises on a capacity or species flag
    log(f"[large {prec}] largest neighbour count seen {mx} (capacity {CAP})")
    assert mx >= max(r["max_rad"] for r in refs.values())
    for k, n in enumerate(SIZES):
        a, z = int(b.offsets[k]), int(b.offsets[k + 1])
        if prec == "fp32":
            tol = (FP32_E_ATOM, FP32_E_ATOM, FP32_F)
        else:
            tol = (None, BF16_E_PER_ATOM, BF16_F)
        _compare(f"large {prec}", n, g["energy"][k], g["e_atom"][a:z], g["forces"][a:z], g["virial"][k],
                 refs[n], b.coords[a:z], *tol)
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_dense_solutes_served_match_oracle(spec, oracle_lib, om, solutes, prec):
    """The large solutes as requests of the native server (capacity 640,
    1 A skin), between small ones: three random-walk steps each; the last
    step of each large request matches the oracle at the coordinates it was
    evaluated at, and no capacity flag is raised."""
    from paper_2207_14276_amd import NNPModel
    from paper_2207_14276_amd.serve import Request, Server, replay
    m = NNPModel(spec, prec)
    small = [synth.water_box(20, seed=71), synth.random_solute(np.random.default_rng(72), 90, 1.2 * 90 ** (1 / 3),
                                                                synth.CONFIG2_PROBS)]
    systems = [small[0], solutes[2000], small[1], solutes[5000]]
    reqs = [Request(s.coords, s.species, s.box, 3, 0.01, seed=500 + k) for k, s in enumerate(systems)]
    srv = Server(m, slots=8000, capacity=CAP, skin=1.0)
    rep = replay(srv, [(0.0, r) for r in reqs])
    srv.close()
    m.status()
    tol = (FP32_E_ATOM, FP32_F) if prec == "fp32" else (BF16_E_PER_ATOM, BF16_F)
    for rid in (1, 3):
        res, s = rep.results[rid], systems[rid]
        E, ea, F, W = oracle_lib.energy_forces(res.coords, s.species, s.box, om)
        de = abs(float(res.energies[-1]) - E) / s.n
        df = float(np.abs(res.forces - F).max())
        log(f"[large served {prec} n={s.n}] |dE_s|/N={de:.3e} max|dF|={df:.3e}")
        assert de <= tol[0]
        assert df <= tol[1]
    m.close()
