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


def run_gpu(model, batch, virial=True, forces=True, check=True):
    c, s, b, o = to_dev(batch)
    r = model.energy_forces(c, s, b, o, forces=forces, virial=virial and forces,
                            atom_energy=True, check=check)
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


def virial_bound(coords, box, f_gpu, f_ref, rc=5.1, w_ref=None):
    """Bound on max |W_gpu - W_ref| of one system derived from its force
    error.  Non-periodic: W = sum_k (r_k - c) (x) F_k for any centre c (the
    pair terms d (x) dE/dd regroup per atom and the net force is zero), so
    |dW_ab| <= sum_k |r_ka - c_a| |dF_kb|, plus float32 rounding of the
    per-centre sums (2e-6 of the same sum over |F|).  Periodic: the lattice
    images break that identity; each atom's share of W is a sum of pair terms
    with lever arms below the cutoff, bounded by rc times its force error.
    Pair terms whose force contributions cancel (an atom and its own images:
    zero net force) still add up in W, so their float32 rounding is bounded
    separately: ~20 roundings of 2^-24 per pair derivative and its sum give
    ~1.2e-6 of |W|; 1e-5 of max |W_ref| is allowed."""
    x = np.asarray(coords, np.float64)
    df = np.abs(np.asarray(f_gpu, np.float64) - np.asarray(f_ref, np.float64))
    fr = np.abs(np.asarray(f_ref, np.float64))
    if box is not None and np.all(np.asarray(box) > 0):
        lever = np.full_like(x, rc)
    else:
        lever = np.abs(x - x.mean(0))
    main = float((lever.T @ df).max())
    slack = 2e-6 * float((lever.T @ fr).max()) + 1e-9 * len(x)
    if w_ref is not None:
        slack += 1e-5 * float(np.abs(np.asarray(w_ref, np.float64)).max())
    return main + slack
