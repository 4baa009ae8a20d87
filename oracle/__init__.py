"""FP64 CPU oracle for the ANI-style energy/force path (ctypes shim).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  The GPU library never
imports, links or calls anything here, and this module never touches the GPU
library.  The arithmetic lives in nnp_oracle.c (plain C, float64, OpenMP over
centre atoms); this file only marshals numpy arrays.

Inputs are a `synth.ModelSpec` (hyper-parameters + float32 weights, read in
float64) and float32 coordinates, also read exactly in float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnp_oracle.c")
_LIB = os.path.join(_HERE, "libnnp_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _AevParams(C.Structure):
    _fields_ = [("n_species", C.c_int),
                ("rc_rad", C.c_double), ("eta_rad", C.c_double),
                ("n_shf_rad", C.c_int), ("shf_rad", C.POINTER(C.c_double)),
                ("rc_ang", C.c_double), ("eta_ang", C.c_double), ("zeta", C.c_double),
                ("n_shf_ang", C.c_int), ("shf_ang", C.POINTER(C.c_double)),
                ("n_shf_z", C.c_int), ("shf_z", C.POINTER(C.c_double)),
                ("radial_scale", C.c_double)]


class _DpParams(C.Structure):
    _fields_ = [("n_species", C.c_int), ("rc", C.c_double), ("sel", C.POINTER(C.c_int))]


class _Model(C.Structure):
    _fields_ = [("aev", _AevParams),
                ("n_ensemble", C.c_int),
                ("n_layers", C.POINTER(C.c_int)),
                ("widths", C.POINTER(C.c_int)),
                ("weights", C.POINTER(C.c_double)),
                ("celu_alpha", C.c_double),
                ("kind", C.c_int),
                ("dp", _DpParams)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        lib.orc_aev_dim.argtypes = [C.POINTER(_AevParams)]
        lib.orc_aev.argtypes = [C.c_int, dp, ip, dp, C.POINTER(_AevParams), dp]
        lib.orc_neighbours.argtypes = [C.c_int, dp, dp, C.c_double, C.c_int, C.c_int, ip, ip]
        lib.orc_energy_forces.argtypes = [C.c_int, dp, ip, dp, C.POINTER(_Model), dp, dp, dp, dp]
        lib.orc_sampled.argtypes = [C.c_int, dp, ip, dp, C.POINTER(_Model), C.c_int, ip, dp, dp]
        lib.orc_dp_dim.argtypes = [C.POINTER(_DpParams)]
        lib.orc_dp_descriptor.argtypes = [C.c_int, dp, ip, dp, C.POINTER(_DpParams), dp]
        lib.orc_net_energy.argtypes = [C.POINTER(_Model), C.c_int, C.c_int, dp, dp]
        lib.orc_net_energy.restype = C.c_double
        lib.orc_threads.restype = C.c_int
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = C.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""


def _aev_struct(p: dict, keep: _Keep) -> _AevParams:
    keep.sr = np.ascontiguousarray(p["shf_rad"], dtype=np.float64)
    keep.sa = np.ascontiguousarray(p["shf_ang"], dtype=np.float64)
    keep.sz = np.ascontiguousarray(p["shf_z"], dtype=np.float64)
    return _AevParams(int(p["n_species"]), float(p["rc_rad"]), float(p["eta_rad"]),
                      len(keep.sr), _dp(keep.sr),
                      float(p["rc_ang"]), float(p["eta_ang"]), float(p["zeta"]),
                      len(keep.sa), _dp(keep.sa), len(keep.sz), _dp(keep.sz),
                      float(p.get("radial_scale", 0.25)))


def _dp_struct(p: dict, keep: _Keep) -> _DpParams:
    keep.sel = np.ascontiguousarray(p["sel"], dtype=np.int32)
    return _DpParams(int(p["n_species"]), float(p["rc"]), _ip(keep.sel))


class OracleModel:
    """float64 copy of a ModelSpec laid out for the C oracle (AEV or
    DeepPot-style descriptor, by spec.aev["kind"])."""

    def __init__(self, spec):
        self.spec = spec
        self._keep = _Keep()
        is_dp = spec.aev.get("kind") == "dp"
        if is_dp:
            self.aev_params = _AevParams()
            self.aev_params.n_species = int(spec.aev["n_species"])
            self.dp_params = _dp_struct(spec.aev, self._keep)
        else:
            self.aev_params = _aev_struct(spec.aev, self._keep)
            self.dp_params = _DpParams()
        self.n_layers = np.array([len(w) - 1 for w in spec.widths], dtype=np.int32)
        self.widths = np.concatenate([np.array(w, dtype=np.int32) for w in spec.widths])
        self.weights = np.ascontiguousarray(spec.weights, dtype=np.float64)
        self.struct = _Model(self.aev_params, int(spec.n_ensemble), _ip(self.n_layers),
                             _ip(self.widths), _dp(self.weights), float(spec.celu_alpha),
                             1 if is_dp else 0, self.dp_params)
        lib = _load()
        self.dim = lib.orc_dp_dim(C.byref(self.dp_params)) if is_dp else lib.orc_aev_dim(C.byref(self.aev_params))


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int) -> int:
    """Threads for later calls (timing only); returns the previous count."""
    return int(_load().orc_set_threads(int(n)))


def _sys_arrays(coords, species, box):
    x = np.ascontiguousarray(np.asarray(coords, dtype=np.float32).astype(np.float64).reshape(-1, 3))
    s = np.ascontiguousarray(species, dtype=np.int32)
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float32).astype(np.float64).reshape(3))
    return x, s, b


def aev(coords, species, box, params: dict) -> np.ndarray:
    """AEV of every atom of one system, [n, D] float64."""
    lib = _load()
    keep = _Keep()
    ap = _aev_struct(params, keep)
    x, s, b = _sys_arrays(coords, species, box)
    D = lib.orc_aev_dim(C.byref(ap))
    out = np.zeros((len(s), D), dtype=np.float64)
    if len(s):
        rc = lib.orc_aev(len(s), _dp(x), _ip(s), _dp(b), C.byref(ap), _dp(out))
        assert rc == 0
    return out


def neighbours(coords, box, rc: float, i: int):
    """Brute-force neighbours of atom i: list of (j, (nx, ny, nz))."""
    lib = _load()
    x, _, b = _sys_arrays(coords, np.zeros(len(coords), np.int32), box)
    cap = 1024
    while True:
        js = np.zeros(cap, np.int32)
        im = np.zeros(3 * cap, np.int32)
        cnt = lib.orc_neighbours(len(x), _dp(x), _dp(b), float(rc), int(i), cap, _ip(js), _ip(im))
        if cnt <= cap:
            break
        cap = cnt
    return [(int(js[e]), tuple(int(v) for v in im[3 * e:3 * e + 3])) for e in range(cnt)]


def energy_forces(coords, species, box, model: OracleModel, forces: bool = True,
                  virial: bool = True):
    """One system: (E_total, e_atom[n], F[n,3] or None, W[3,3] or None), float64."""
    lib = _load()
    x, s, b = _sys_arrays(coords, species, box)
    n = len(s)
    e_atom = np.zeros(n, np.float64)
    E = np.zeros(1, np.float64)
    F = np.zeros((n, 3), np.float64) if forces else None
    W = np.zeros(9, np.float64) if virial else None
    if n:
        rc = lib.orc_energy_forces(n, _dp(x), _ip(s), _dp(b), C.byref(model.struct),
                                   _dp(e_atom), _dp(E), _dp(F), _dp(W))
        assert rc == 0
    return float(E[0]), e_atom, F, (W.reshape(3, 3) if W is not None else None)


def batch_energy_forces(batch, model: OracleModel, systems=None, forces: bool = True,
                        virial: bool = True):
    """Per-system oracle over a synth.Batch (optionally a subset of systems).

    Returns dict with energy[S'] and per-system e_atom / forces / virial lists.
    """
    idx = range(batch.n_systems) if systems is None else systems
    out = {"systems": list(idx), "energy": [], "e_atom": [], "forces": [], "virial": []}
    for k in idx:
        a, e = int(batch.offsets[k]), int(batch.offsets[k + 1])
        E, ea, F, W = energy_forces(batch.coords[a:e], batch.species[a:e], batch.boxes[k],
                                    model, forces, virial)
        out["energy"].append(E)
        out["e_atom"].append(ea)
        out["forces"].append(F)
        out["virial"].append(W)
    out["energy"] = np.array(out["energy"])
    return out


def sampled(coords, species, box, model: OracleModel, targets):
    """Atomic energies and forces of the given atoms only (exact, local)."""
    lib = _load()
    x, s, b = _sys_arrays(coords, species, box)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    e = np.zeros(len(t), np.float64)
    f = np.zeros((len(t), 3), np.float64)
    rc = lib.orc_sampled(len(s), _dp(x), _ip(s), _dp(b), C.byref(model.struct), len(t),
                         _ip(t), _dp(e), _dp(f))
    assert rc == 0
    return e, f


def net_energy(model: OracleModel, member: int, species: int, G):
    """One network on one AEV: (E, dE/dG)."""
    lib = _load()
    G = np.ascontiguousarray(G, dtype=np.float64)
    g = np.zeros(model.dim, np.float64)
    E = lib.orc_net_energy(C.byref(model.struct), int(member), int(species), _dp(G), _dp(g))
    return float(E), g


def dp_descriptor(coords, species, box, p: dict):
    """DeepPot-style descriptor of every atom: float64 [n, 4 * sum(sel)]."""
    lib = _load()
    x, s, b = _sys_arrays(coords, species, box)
    keep = _Keep()
    st = _dp_struct(p, keep)
    D = lib.orc_dp_dim(C.byref(st))
    out = np.zeros((len(s), D), np.float64)
    if len(s):
        assert lib.orc_dp_descriptor(len(s), _dp(x), _ip(s), _dp(b), C.byref(st), _dp(out)) == 0
    return out
