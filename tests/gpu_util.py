"""Helpers for the GPU tests: run the HIP path through the C ABI on synthetic
inputs and compare with the FP64 oracle."""
import sys

import numpy as np
import torch

import synth

# Tolerances (kcal/mol, kcal/mol/A) of the float32 path and of the path whose
# dense layers take bfloat16 operands.
FP32_E_ATOM = 1e-5
FP32_F = 1e-3
BF16_E_PER_ATOM = 1e-2
BF16_F = 5e-2


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(batch, device="cuda"):
    return (torch.as_tensor(batch.coords, device=device),
            torch.as_tensor(batch.species, device=device),
            batch.boxes, batch.offsets)


def run_gpu(model, batch, virial=True, forces=True):
    c, s, b, o = to_dev(batch)
    r = model.energy_forces(c, s, b, o, forces=forces, virial=virial and forces,
                            atom_energy=True, check=True)
    torch.cuda.synchronize()
    out = {"energy": r.energy.cpu().numpy(), "e_atom": r.atom_energy.cpu().numpy().astype(np.float64)}
    if forces:
        out["forces"] = r.forces.cpu().numpy().astype(np.float64)
    if virial and forces:
        out["virial"] = r.virial.cpu().numpy()
    return out


def compare_system(gpu, ora, k, batch, label, e_atom_tol, f_tol, e_sys_per_atom_tol=None):
    a, e = int(batch.offsets[k]), int(batch.offsets[k + 1])
    n = e - a
    de_atom = np.abs(gpu["e_atom"][a:e] - ora["e_atom"][k]).max() if n else 0.0
    de_sys = abs(gpu["energy"][k] - ora["energy"][k]) / max(n, 1)
    df = np.abs(gpu["forces"][a:e] - ora["forces"][k]).max() if n and "forces" in gpu else 0.0
    return de_atom, de_sys, df
