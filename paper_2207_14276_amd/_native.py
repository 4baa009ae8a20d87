"""ctypes binding of libnnp.so (include/nnp.h), argument marshalling only.

The functions here carry the C names.  Every step of the computation runs in
the HIP library; there is no CPU fallback: if the library is missing this
module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libnnp.so")

NNP_OK = 0
NNP_EINVAL = -1
NNP_ENOMEM = -2
NNP_ECAPACITY = -3
NNP_EDEVICE = -4
NNP_ESPECIES = -5
NNP_EUNSUPPORTED = -6
NNP_FP32 = 0
NNP_BF16 = 1

_ERR_NAMES = {NNP_EINVAL: "EINVAL", NNP_ENOMEM: "ENOMEM", NNP_ECAPACITY: "ECAPACITY",
              NNP_EDEVICE: "EDEVICE", NNP_ESPECIES: "ESPECIES",
              NNP_EUNSUPPORTED: "EUNSUPPORTED"}


class NNPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nnp error {_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class nnp_aev_params(C.Structure):
    _fields_ = [("n_species", C.c_int),
                ("rc_rad", C.c_float), ("eta_rad", C.c_float),
                ("n_shf_rad", C.c_int), ("shf_rad", C.POINTER(C.c_float)),
                ("rc_ang", C.c_float), ("eta_ang", C.c_float), ("zeta", C.c_float),
                ("n_shf_ang", C.c_int), ("shf_ang", C.POINTER(C.c_float)),
                ("n_shf_z", C.c_int), ("shf_z", C.POINTER(C.c_float)),
                ("radial_scale", C.c_float)]


class nnp_model_desc(C.Structure):
    _fields_ = [("aev", nnp_aev_params),
                ("n_ensemble", C.c_int),
                ("n_layers", C.POINTER(C.c_int)),
                ("widths", C.POINTER(C.c_int)),
                ("weights", C.POINTER(C.c_float)),
                ("celu_alpha", C.c_float),
                ("precision", C.c_int)]


class nnp_dp_params(C.Structure):
    _fields_ = [("n_species", C.c_int), ("rc", C.c_float), ("sel", C.POINTER(C.c_int))]


class nnp_dp_model_desc(C.Structure):
    _fields_ = [("dp", nnp_dp_params),
                ("n_ensemble", C.c_int),
                ("n_layers", C.POINTER(C.c_int)),
                ("widths", C.POINTER(C.c_int)),
                ("weights", C.POINTER(C.c_float)),
                ("celu_alpha", C.c_float),
                ("precision", C.c_int)]


class nnp_server_opts(C.Structure):
    _fields_ = [("slots", C.c_int64), ("nbr_capacity", C.c_int), ("skin", C.c_float),
                ("max_batch_atoms", C.c_int64), ("max_active", C.c_int),
                ("hbm_budget", C.c_uint64), ("use_graphs", C.c_int)]


class nnp_request(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("coords", C.POINTER(C.c_float)),
                ("species", C.POINTER(C.c_int32)), ("box", C.c_float * 3),
                ("n_steps", C.c_int), ("sigma", C.c_float), ("seed", C.c_uint64)]


class nnp_server_counters(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("atom_evals", C.c_int64), ("queued", C.c_int64),
                ("active", C.c_int64), ("max_batch_atoms", C.c_int64),
                ("max_batch_seen", C.c_int64), ("device_bytes", C.c_uint64),
                ("list_builds", C.c_int64), ("graph_captures", C.c_int64),
                ("graph_replays", C.c_int64), ("host_launch_s", C.c_double)]


EXPORTS = ["nnp_create", "nnp_destroy", "nnp_reserve", "nnp_energy_forces", "nnp_debug_aev",
           "nnp_energy_forces_noalloc",
           "nnp_debug_neighbors", "nnp_status", "nnp_aev_dim", "nnp_last_error",
           "nnp_set_timing", "nnp_stage_timings", "nnp_nlist_create", "nnp_nlist_destroy",
           "nnp_energy_forces_nlist", "nnp_nlist_builds", "nnp_autotune", "nnp_tuning",
           "nnp_energy_forces_pairs", "nnp_bar", "nnp_create_dp",
           "nnp_server_create", "nnp_server_destroy", "nnp_server_clock", "nnp_server_submit",
           "nnp_server_step", "nnp_server_drain", "nnp_server_poll", "nnp_server_result",
           "nnp_server_stats",
           "nnp_sched_create", "nnp_sched_destroy", "nnp_sched_submit", "nnp_sched_admit",
           "nnp_sched_launch", "nnp_sched_complete", "nnp_sched_job", "nnp_sched_info",
           "nnp_sched_fail"]

_lib = None


def load():
    """Loads libnnp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2207_14276_amd.build` (there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
    fp = C.POINTER(C.c_float)
    lib.nnp_create.argtypes = [C.POINTER(nnp_model_desc), C.c_int, C.POINTER(C.c_void_p)]
    lib.nnp_create_dp.argtypes = [C.POINTER(nnp_dp_model_desc), C.c_int, C.POINTER(C.c_void_p)]
    lib.nnp_destroy.argtypes = [vp]
    lib.nnp_destroy.restype = None
    lib.nnp_reserve.argtypes = [vp, C.c_int64, C.c_int, C.c_int]
    lib.nnp_energy_forces.argtypes = [vp, C.c_int, i64p, vp, vp, fp, vp, vp, vp, vp, vp]
    lib.nnp_energy_forces_noalloc.argtypes = [vp, C.c_int, i64p, vp, vp, fp, vp, vp, vp, vp, vp]
    lib.nnp_debug_aev.argtypes = [vp, C.c_int, i64p, vp, vp, fp, vp, vp]
    lib.nnp_debug_neighbors.argtypes = [vp, C.c_int, i64p, vp, vp, fp, vp, vp, C.c_int, vp]
    lib.nnp_status.argtypes = [vp, vp, C.POINTER(C.c_int)]
    lib.nnp_aev_dim.argtypes = [vp]
    lib.nnp_last_error.restype = C.c_char_p
    lib.nnp_set_timing.argtypes = [vp, C.c_int]
    lib.nnp_stage_timings.argtypes = [vp, fp, C.POINTER(C.c_char_p), C.c_int]
    lib.nnp_nlist_create.argtypes = [vp, C.c_int64, C.c_int, C.c_float, C.POINTER(C.c_void_p)]
    lib.nnp_nlist_destroy.argtypes = [vp]
    lib.nnp_nlist_destroy.restype = None
    lib.nnp_energy_forces_nlist.argtypes = [vp, vp, C.c_int, i64p, i64p, C.POINTER(C.c_int32), vp,
                                            vp, fp, vp, vp, vp, vp, vp]
    lib.nnp_nlist_builds.argtypes = [vp, vp, i64p]
    dpp = C.POINTER(C.c_double)
    lib.nnp_bar.argtypes = [C.c_int64, dpp, dpp, C.c_int64, dpp, dpp, dpp, dpp]
    lib.nnp_energy_forces_pairs.argtypes = [vp, C.c_int64, vp, vp, fp, C.c_int64, vp, vp, C.c_int, vp,
                                            vp, vp, vp, vp, vp]
    lib.nnp_autotune.argtypes = [vp, C.c_int, i64p, vp, vp, fp, vp]
    lib.nnp_tuning.argtypes = [vp, C.POINTER(C.c_int), C.c_int]
    dp, i32p, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int)
    lib.nnp_server_create.argtypes = [vp, C.POINTER(nnp_server_opts), C.POINTER(C.c_void_p)]
    lib.nnp_server_destroy.argtypes = [vp]
    lib.nnp_server_destroy.restype = None
    lib.nnp_server_clock.argtypes = [vp]
    lib.nnp_server_clock.restype = C.c_double
    lib.nnp_server_submit.argtypes = [vp, C.POINTER(nnp_request), C.c_double, i64p]
    lib.nnp_server_step.argtypes = [vp, vp, i64p]
    lib.nnp_server_drain.argtypes = [vp]
    lib.nnp_server_poll.argtypes = [vp, i64p, C.c_int, ip]
    lib.nnp_server_result.argtypes = [vp, C.c_int64, dp, fp, fp, dp]
    lib.nnp_server_stats.argtypes = [vp, C.POINTER(nnp_server_counters)]
    lib.nnp_sched_create.argtypes = [C.c_int64, C.c_int64, C.c_int, C.POINTER(C.c_void_p)]
    lib.nnp_sched_destroy.argtypes = [vp]
    lib.nnp_sched_destroy.restype = None
    lib.nnp_sched_submit.argtypes = [vp, C.c_int64, C.c_int, C.c_int, C.c_double]
    lib.nnp_sched_admit.argtypes = [vp, C.c_double, i64p, i64p, C.c_int, ip]
    lib.nnp_sched_launch.argtypes = [vp, i64p, i64p, i32p, i32p, C.c_int, ip]
    lib.nnp_sched_complete.argtypes = [vp, C.c_int64, C.c_double, ip]
    lib.nnp_sched_fail.argtypes = [vp, C.c_int64, C.c_double]
    lib.nnp_sched_job.argtypes = [vp, C.c_int64, dp, i64p, i32p]
    lib.nnp_sched_info.argtypes = [vp, i64p]
    _lib = lib
    return lib


def check(rc):
    if rc < 0:
        raise NNPError(rc, load().nnp_last_error().decode())
    return rc


def last_error() -> str:
    return load().nnp_last_error().decode()
