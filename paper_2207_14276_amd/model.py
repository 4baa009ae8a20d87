"""Python face of the library: a model handle and a torch.autograd.Function.

PyTorch provides device memory and streams only: inputs and outputs are torch
tensors whose device addresses go straight through the C ABI (the paper's
raw-address interface, section "A General Machine Learning Platform"), and
the library enqueues its kernels on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as nat


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _stream_handle(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Result:
    energy: torch.Tensor                 # [S] float64
    forces: torch.Tensor | None = None   # [N, 3] float32
    virial: torch.Tensor | None = None   # [S, 3, 3] float64
    atom_energy: torch.Tensor | None = None  # [N] float32


class NNPModel:
    """A network set on one GPU.

    `spec` carries the descriptor hyper-parameters (dict `aev`: the AEV's, or
    a DeepPot-style descriptor's with kind "dp", cutoff rc and per-species
    capacities sel), `n_ensemble`, per-species `widths`, float32 `weights`
    (member, species, layer; W[out][in] then b[out]) and `celu_alpha`.
    `precision` is "fp32" or "bf16" (dense layers with bfloat16 operands and
    float32 accumulation).
    """

    def __init__(self, spec, precision: str = "fp32", device=None):
        lib = nat.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.spec = spec
        self.precision = precision
        p = spec.aev
        keep = {
            "nl": np.array([len(w) - 1 for w in spec.widths], np.int32),
            "w": np.concatenate([np.array(w, np.int32) for w in spec.widths]),
            "weights": np.ascontiguousarray(spec.weights, np.float32),
        }
        nets = (int(spec.n_ensemble), keep["nl"].ctypes.data_as(C.POINTER(C.c_int)),
                keep["w"].ctypes.data_as(C.POINTER(C.c_int)), _fptr(keep["weights"]),
                float(spec.celu_alpha), nat.NNP_BF16 if precision == "bf16" else nat.NNP_FP32)
        h = C.c_void_p()
        if p.get("kind") == "dp":
            keep["sel"] = np.ascontiguousarray(p["sel"], np.int32)
            dp = nat.nnp_dp_params(int(p["n_species"]), float(p["rc"]),
                                   keep["sel"].ctypes.data_as(C.POINTER(C.c_int)))
            desc = nat.nnp_dp_model_desc(dp, *nets)
            create = lib.nnp_create_dp
        else:
            keep["sr"] = np.ascontiguousarray(p["shf_rad"], np.float32)
            keep["sa"] = np.ascontiguousarray(p["shf_ang"], np.float32)
            keep["sz"] = np.ascontiguousarray(p["shf_z"], np.float32)
            aev = nat.nnp_aev_params(int(p["n_species"]), float(p["rc_rad"]), float(p["eta_rad"]),
                                     len(keep["sr"]), _fptr(keep["sr"]),
                                     float(p["rc_ang"]), float(p["eta_ang"]), float(p["zeta"]),
                                     len(keep["sa"]), _fptr(keep["sa"]),
                                     len(keep["sz"]), _fptr(keep["sz"]),
                                     float(p.get("radial_scale", 0.25)))
            desc = nat.nnp_model_desc(aev, *nets)
            create = lib.nnp_create
        nat.check(create(C.byref(desc), int(self.device.index), C.byref(h)))
        self._h = h
        self.aev_dim = lib.nnp_aev_dim(h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            nat.load().nnp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def reserve(self, max_atoms: int, max_systems: int = 1, nbr_capacity: int = 0):
        with torch.cuda.device(self.device):
            nat.check(nat.load().nnp_reserve(self._h, int(max_atoms), int(max_systems),
                                             int(nbr_capacity)))

    # ---------------------------------------------------------------- inputs
    def _inputs(self, coords, species, boxes, offsets):
        coords = coords.to(self.device, torch.float32).contiguous()
        species = species.to(self.device, torch.int32).contiguous()
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        bx = boxes.detach().cpu().numpy() if torch.is_tensor(boxes) else np.asarray(boxes)
        bx = np.ascontiguousarray(bx, dtype=np.float32).reshape(-1, 3)
        S = len(offs) - 1
        if bx.shape[0] != S:
            raise ValueError(f"boxes has {bx.shape[0]} rows for {S} systems")
        return coords, species, bx, offs, S

    def energy_forces(self, coords, species, boxes, offsets, forces: bool = True,
                      virial: bool = False, atom_energy: bool = False, check: bool = False,
                      out: Result | None = None) -> Result:
        """Energies [S] (float64) and, if asked, forces [N,3], virials [S,3,3]
        and atomic energies [N].  Asynchronous on the current stream unless
        check=True, which waits and raises on a device flag (neighbour
        overflow retries once with a larger capacity)."""
        coords, species, bx, offs, S = self._inputs(coords, species, boxes, offsets)
        N = int(offs[-1])
        if out is None:
            out = Result(energy=torch.empty(S, dtype=torch.float64, device=self.device))
            if forces:
                out.forces = torch.empty((N, 3), dtype=torch.float32, device=self.device)
            if virial:
                out.virial = torch.empty((S, 3, 3), dtype=torch.float64, device=self.device)
            if atom_energy:
                out.atom_energy = torch.empty(N, dtype=torch.float32, device=self.device)
        lib = nat.load()
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        with torch.cuda.device(self.device):
            st = _stream_handle(self.device)
            for attempt in range(2):
                nat.check(lib.nnp_energy_forces(
                    self._h, S, offs.ctypes.data_as(C.POINTER(C.c_int64)), ptr(coords),
                    ptr(species), _fptr(bx), ptr(out.energy), ptr(out.forces), ptr(out.virial),
                    ptr(out.atom_energy), st))
                if not check:
                    break
                mx = C.c_int()
                rc = lib.nnp_status(self._h, st, C.byref(mx))
                if rc == nat.NNP_ECAPACITY and attempt == 0:
                    self.reserve(N, S, min(1024, max(int(mx.value * 1.25) + 4, 64)))
                    continue
                nat.check(rc)
                break
        return out

    def energy_forces_pairs(self, coords, species, box, pairs, shifts=None, mask=None,
                            half: bool = True, forces: bool = True, virial: bool = False,
                            atom_energy: bool = False, check: bool = False,
                            out: Result | None = None) -> Result:
        """One system from the caller's pair list (nnp_energy_forces_pairs):
        `pairs` [P, 2] int32 (i, j), `shifts` [P, 3] int32 lattice shifts or
        None, `mask` [N] bool/uint8 ML region or None (all atoms), `box` [3]
        (zeros: non-periodic).  Energy [1] float64, forces [N, 3], virial
        [1, 3, 3], atomic energies [N] as in energy_forces.  check=True waits
        and raises on a device flag (a neighbour overflow retries once with a
        larger capacity)."""
        coords = coords.to(self.device, torch.float32).contiguous()
        species = species.to(self.device, torch.int32).contiguous()
        N = int(coords.shape[0])
        pairs = pairs.to(self.device, torch.int32).contiguous()
        P = int(pairs.shape[0])
        if pairs.dim() != 2 or pairs.shape[1] != 2:
            raise ValueError("pairs must be [P, 2]")
        if shifts is not None:
            shifts = shifts.to(self.device, torch.int32).contiguous()
            if tuple(shifts.shape) != (P, 3):
                raise ValueError("shifts must be [P, 3]")
        if mask is not None:
            mask = mask.to(self.device, torch.uint8).contiguous()
            if tuple(mask.shape) != (N,):
                raise ValueError("mask must be [N]")
        bx = box.detach().cpu().numpy() if torch.is_tensor(box) else np.asarray(box)
        bx = np.ascontiguousarray(bx, dtype=np.float32).reshape(3)
        if out is None:
            out = Result(energy=torch.empty(1, dtype=torch.float64, device=self.device))
            if forces:
                out.forces = torch.empty((N, 3), dtype=torch.float32, device=self.device)
            if virial:
                out.virial = torch.empty((1, 3, 3), dtype=torch.float64, device=self.device)
            if atom_energy:
                out.atom_energy = torch.empty(N, dtype=torch.float32, device=self.device)
        lib = nat.load()
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        with torch.cuda.device(self.device):
            st = _stream_handle(self.device)
            for attempt in range(2):
                nat.check(lib.nnp_energy_forces_pairs(
                    self._h, N, ptr(coords), ptr(species), _fptr(bx), P, ptr(pairs), ptr(shifts),
                    1 if half else 0, ptr(mask), ptr(out.energy), ptr(out.forces), ptr(out.virial),
                    ptr(out.atom_energy), st))
                if not check:
                    break
                mx = C.c_int()
                rc = lib.nnp_status(self._h, st, C.byref(mx))
                if rc == nat.NNP_ECAPACITY and attempt == 0:
                    self.reserve(N, 1, min(1024, max(int(mx.value * 1.25) + 4, 64)))
                    continue
                nat.check(rc)
                break
        return out

    def autotune(self, coords, species, boxes, offsets) -> dict:
        """Picks the launch shapes (AEV waves per workgroup, GEMM column-tile
        widths) that run this batch fastest; they stay with the model.
        Returns {site: value} for the sites that were tuned."""
        coords, species, bx, offs, S = self._inputs(coords, species, boxes, offsets)
        with torch.cuda.device(self.device):
            nat.check(nat.load().nnp_autotune(
                self._h, S, offs.ctypes.data_as(C.POINTER(C.c_int64)), C.c_void_p(coords.data_ptr()),
                C.c_void_p(species.data_ptr()), _fptr(bx), _stream_handle(self.device)))
        return self.tuning()

    def tuning(self) -> dict:
        vals = (C.c_int * 32)()
        n = nat.check(nat.load().nnp_tuning(self._h, vals, 32))
        names = {0: "aev_fwd_waves", 1: "aev_bwd_waves", 18: "gemm_dEdG_tn", 19: "chain_waves"}
        out = {}
        for q in range(n):
            if vals[q]:
                name = names.get(q) or (f"gemm_fwd{q - 2}_tn" if q < 10 else f"gemm_bwd{q - 10}_tn")
                out[name] = int(vals[q])
        return out

    def status(self):
        mx = C.c_int()
        with torch.cuda.device(self.device):
            nat.check(nat.load().nnp_status(self._h, _stream_handle(self.device), C.byref(mx)))
        return int(mx.value)

    def aev(self, coords, species, boxes, offsets) -> torch.Tensor:
        coords, species, bx, offs, S = self._inputs(coords, species, boxes, offsets)
        N = int(offs[-1])
        out = torch.empty((N, self.aev_dim), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            nat.check(nat.load().nnp_debug_aev(
                self._h, S, offs.ctypes.data_as(C.POINTER(C.c_int64)),
                C.c_void_p(coords.data_ptr()), C.c_void_p(species.data_ptr()), _fptr(bx),
                C.c_void_p(out.data_ptr()), _stream_handle(self.device)))
        return out

    def neighbors(self, coords, species, boxes, offsets, capacity: int = 256):
        """(counts [N], entries [N, capacity, 4] = (j, image x, y, z))."""
        coords, species, bx, offs, S = self._inputs(coords, species, boxes, offsets)
        N = int(offs[-1])
        cnt = torch.empty(N, dtype=torch.int32, device=self.device)
        ent = torch.full((N, capacity, 4), -1, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            nat.check(nat.load().nnp_debug_neighbors(
                self._h, S, offs.ctypes.data_as(C.POINTER(C.c_int64)),
                C.c_void_p(coords.data_ptr()), C.c_void_p(species.data_ptr()), _fptr(bx),
                C.c_void_p(cnt.data_ptr()), C.c_void_p(ent.data_ptr()), int(capacity),
                _stream_handle(self.device)))
        return cnt, ent

    STAGES = ("ingest", "cells", "neighbours", "buckets", "aev_fwd", "mlp", "aev_bwd", "reduce")

    def set_timing(self, on: bool = True, stage: str = None):
        """Stage timing on (every stage, or only `stage`, by its name) or off."""
        mode = 0 if not on else (1 if stage is None else 2 + self.STAGES.index(stage))
        nat.check(nat.load().nnp_set_timing(self._h, mode))

    def stage_timings(self) -> dict:
        """Mean ms per recorded call of each recorded stage."""
        ms = (C.c_float * 16)()
        names = (C.c_char_p * 16)()
        k = nat.check(nat.load().nnp_stage_timings(self._h, ms, names, 16))
        return {names[q].decode(): float(ms[q]) for q in range(k) if ms[q] >= 0.0}


class NeighborPool:
    """Persistent device-resident neighbour lists (nnp_nlist): `slots` atom
    slots, lists built with the descriptor cutoff + skin and reused until an atom of
    the system has moved more than skin / 2 since its last build."""

    def __init__(self, model: NNPModel, slots: int, capacity: int = 256, skin: float = 1.0):
        self.model = model
        self.slots = int(slots)
        self.capacity = int(capacity)
        self.skin = float(skin)
        h = C.c_void_p()
        with torch.cuda.device(model.device):
            nat.check(nat.load().nnp_nlist_create(model.handle, self.slots, self.capacity,
                                                  self.skin, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            nat.load().nnp_nlist_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def builds(self) -> int:
        b = C.c_int64()
        with torch.cuda.device(self.model.device):
            nat.check(nat.load().nnp_nlist_builds(self._h, _stream_handle(self.model.device), C.byref(b)))
        return int(b.value)

    def energy_forces(self, coords, species, boxes, offsets, slots, rebuild=None,
                      forces: bool = True, virial: bool = False, atom_energy: bool = False,
                      out: Result | None = None) -> Result:
        """Energies (and forces) of a batch whose system s keeps its list in
        pool slots [slots[s], slots[s] + n_s); rebuild[s] != 0 forces a fresh list."""
        m = self.model
        coords, species, bx, offs, S = m._inputs(coords, species, boxes, offsets)
        N = int(offs[-1])
        sl = np.ascontiguousarray(np.asarray(slots, dtype=np.int64))
        rb = None if rebuild is None else np.ascontiguousarray(np.asarray(rebuild, dtype=np.int32))
        if out is None:
            out = Result(energy=torch.empty(S, dtype=torch.float64, device=m.device))
            if forces:
                out.forces = torch.empty((N, 3), dtype=torch.float32, device=m.device)
            if virial:
                out.virial = torch.empty((S, 3, 3), dtype=torch.float64, device=m.device)
            if atom_energy:
                out.atom_energy = torch.empty(N, dtype=torch.float32, device=m.device)
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        with torch.cuda.device(m.device):
            nat.check(nat.load().nnp_energy_forces_nlist(
                m.handle, self._h, S, offs.ctypes.data_as(C.POINTER(C.c_int64)),
                sl.ctypes.data_as(C.POINTER(C.c_int64)),
                rb.ctypes.data_as(C.POINTER(C.c_int32)) if rb is not None else None,
                ptr(coords), ptr(species), _fptr(bx), ptr(out.energy), ptr(out.forces),
                ptr(out.virial), ptr(out.atom_energy), _stream_handle(m.device)))
        return out


class NNPFunction(torch.autograd.Function):
    """E = NNPFunction.apply(coords, species, boxes, offsets, model) -> [S] float64.

    The forward pass computes energies and forces in one library call; the
    backward pass returns -grad_E[system of atom] * F without another kernel
    pass over the network.  Double backward is not supported.
    """

    @staticmethod
    def forward(ctx, coords, species, boxes, offsets, model: NNPModel):
        res = model.energy_forces(coords, species, boxes, offsets, forces=True)
        offs = np.asarray(offsets, dtype=np.int64)
        counts = torch.as_tensor(np.diff(offs), device=coords.device)
        ctx.save_for_backward(res.forces, counts)
        ctx.coords_dtype = coords.dtype
        return res.energy

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_e):
        forces, counts = ctx.saved_tensors
        g = torch.repeat_interleave(grad_e.to(torch.float32), counts)
        return (-g[:, None] * forces).to(ctx.coords_dtype), None, None, None, None
