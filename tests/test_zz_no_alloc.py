"""The entry point that allocates nothing (nnp_energy_forces_noalloc),
through the C ABI: two calls in a row, the second on a smaller batch, each
against nnp_energy_forces on the same inputs at the float32 and bfloat16
parity bars; a call too large for the fixed scratch is refused before
anything is enqueued, and the model keeps working afterwards."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import BF16_E_PER_ATOM, BF16_F, FP32_E_ATOM, FP32_F, log, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(model, batch):
    from paper_2207_14276_amd import _native as nat
    c, s, bx, o = to_dev(batch)
    S, N = batch.n_systems, batch.n_atoms
    e = torch.empty(S, dtype=torch.float64, device="cuda")
    f = torch.empty((N, 3), dtype=torch.float32, device="cuda")
    w = torch.empty((S, 3, 3), dtype=torch.float64, device="cuda")
    ea = torch.empty(N, dtype=torch.float32, device="cuda")
    offs = np.ascontiguousarray(o, np.int64)
    box = np.ascontiguousarray(bx, np.float32)
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = nat.load().nnp_energy_forces_noalloc(
        model.handle, S, offs.ctypes.data_as(C.POINTER(C.c_int64)), p(c), p(s),
        box.ctypes.data_as(C.POINTER(C.c_float)), p(e), p(f), p(w), p(ea),
        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, e, f, w, ea


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_matches_energy_forces(prec):
    from paper_2207_14276_amd import NNPModel
    from paper_2207_14276_amd import _native as nat
    spec = synth.make_model(0)
    m = NNPModel(spec, prec)
    big = synth.ragged_solutes(24, seed=41)                 # ~1,600 atoms
    small = synth.make_batch([synth.water_box(60, seed=42),  # periodic, then a solute
                              synth.config0()])
    e_tol, f_tol = (FP32_E_ATOM, FP32_F) if prec == "fp32" else (BF16_E_PER_ATOM, BF16_F)
    for label, b in (("first", big), ("second, smaller", small)):
        log(f"[noalloc {prec}] {label} call: {b.n_systems} systems, {b.n_atoms} atoms", )
        rc, e, f, w, ea = _noalloc(m, b)
        assert rc == 0, nat.last_error()
        c, s, bx, o = to_dev(b)
        ref = m.energy_forces(c, s, bx, o, forces=True, virial=True, atom_energy=True, check=True)
        torch.cuda.synchronize()
        m.status()
        n = torch.as_tensor(np.diff(b.offsets), device="cuda", dtype=torch.float64)
        de = float(((e - ref.energy).abs() / n).max())
        df = float((f - ref.forces).abs().max())
        dea = float((ea - ref.atom_energy).abs().max())
        dw = float((w - ref.virial).abs().max())
        log(f"[noalloc {prec}] {label}: |dE|/N={de:.3e} max|dF|={df:.3e} max|dE_i|={dea:.3e} "
            f"max|dW|={dw:.3e} bitwise={bool(torch.equal(f, ref.forces) and torch.equal(e, ref.energy))}")
        assert de <= e_tol
        assert df <= f_tol
        assert dea <= (e_tol if prec == "fp32" else 1e-1)
    # beyond the fixed scratch: refused before anything runs
    huge = synth.make_batch([synth.water_box(4000, seed=43)])
    rc, *_ = _noalloc(m, huge)
    assert rc == nat.NNP_EUNSUPPORTED, rc
    assert "scratch" in nat.last_error()
    rc, e, f, w, ea = _noalloc(m, small)
    assert rc == 0
    torch.cuda.synchronize()
    m.status()
    m.close()
