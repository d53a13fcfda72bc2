"""ctypes binding of libapx.so: structure layouts and function prototypes of apx.h.

Argument marshalling only.  Loading fails loudly when the library has not been built;
there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapx.so")

APX_OK = 0
APX_EINVAL = -1
APX_ENOMEM = -2
APX_EDEVICE = -3
APX_ECAPACITY = -4
APX_ENONFINITE = -5
APX_ERADICAND = -6
APX_FP64 = 0
APX_FP32 = 1
MODE_ADAPTIVE = 0
MODE_FULL_ACE = 1
MODE_EAM = 2

_P = C.c_void_p


class Atoms(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", _P), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("periodic", C.c_int32 * 3), ("frozen", _P)]


class NList(C.Structure):
    _fields_ = [("n", C.c_int64), ("max_nb", C.c_int32), ("count", _P), ("idx", _P), ("r_list", C.c_double)]


class PrecParams(C.Structure):
    _fields_ = [("n_nn", C.c_int32), ("n_buffer", C.c_int32), ("switch_kind", C.c_int32),
                ("flags", C.c_int32), ("csp_lo", C.c_double), ("csp_hi", C.c_double),
                ("r_cut", C.c_double), ("r_lo", C.c_double), ("r_hi", C.c_double)]


EAM_CLOSED, EAM2 = 0, 1


class EamParams(C.Structure):
    _fields_ = [("A", C.c_double), ("alpha", C.c_double), ("beta", C.c_double), ("r0", C.c_double),
                ("r_cut", C.c_double), ("h", C.c_double), ("kind", C.c_int32), ("reserved", C.c_int32),
                ("eam2", C.c_double * 27)]


class AceDesc(C.Structure):
    _fields_ = [("n_max", C.c_int32), ("l_max", C.c_int32), ("r_cut", C.c_double), ("h", C.c_double),
                ("s_a", C.c_double), ("eps", C.c_double), ("W", _P), ("c1", _P), ("c2", _P),
                ("anchored", C.c_int32), ("reserved", C.c_int32), ("anchor", EamParams)]


class ThermoParams(C.Structure):
    _fields_ = [("r_omega", C.c_double), ("omega_max", C.c_int32), ("group_batch", C.c_int32), ("seed", C.c_uint64)]


class MdParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("mass", C.c_double), ("skin", C.c_double), ("max_nb", C.c_int32),
                ("precision_every", C.c_int32), ("ace_precision", C.c_int32), ("mode", C.c_int32),
                ("indenter", C.c_int32), ("avg_samples", C.c_int32), ("ind_radius", C.c_double),
                ("ind_k", C.c_double), ("ind_center", C.c_double * 3), ("ind_velocity", C.c_double * 3),
                ("avg_dw_min", C.c_double), ("avg_window", C.c_int32), ("thermostat", C.c_int32),
                ("thermo", ThermoParams)]


class AvgState(C.Structure):
    _fields_ = [("n_avg", C.c_int32), ("window", C.c_int32), ("samples", C.c_int64), ("dw_min", C.c_double),
                ("csp_ring", _P), ("w_ring", _P)]


class MdStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("precision_updates", C.c_int64),
                ("n_active", C.c_int64), ("e_pot", C.c_double), ("e_kin", C.c_double),
                ("e_indenter", C.c_double), ("ace_atoms", C.c_int64), ("thermo_steps", C.c_int64),
                ("thermo_corrected", C.c_int64), ("thermo_failed", C.c_int64)]


# name -> (restype, argtypes); every symbol declared in include/apx.h
PROTOTYPES = {
    "apx_ctx_create": (C.c_int32, [C.c_int32, _P, C.POINTER(_P)]),
    "apx_ctx_set_stream": (C.c_int32, [_P, _P]),
    "apx_ctx_destroy": (None, [_P]),
    "apx_last_error": (C.c_char_p, [_P]),
    "apx_ctx_synchronize": (C.c_int32, [_P]),
    "apx_version": (C.c_char_p, []),
    "apx_profile_enable": (C.c_int32, [_P, C.c_int32]),
    "apx_profile_count": (C.c_int32, [_P]),
    "apx_profile_entry": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_char_p), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double)]),
    "apx_ace_model_stats": (C.c_int32, [_P, C.POINTER(C.c_int64)]),
    "apx_fp64_functions": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P]),
    "apx_build_neighbors": (C.c_int32, [_P, C.POINTER(Atoms), C.c_double, C.POINTER(NList), C.POINTER(C.c_int32)]),
    "apx_compute_precision": (C.c_int32, [_P, C.POINTER(Atoms), C.POINTER(NList), C.POINTER(PrecParams), _P,
                                          _P, _P, _P, _P, _P, C.POINTER(C.c_int64)]),
    "apx_compute_precision_avg": (C.c_int32, [_P, C.POINTER(Atoms), C.POINTER(NList), C.POINTER(PrecParams),
                                              C.POINTER(AvgState), _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                              C.POINTER(C.c_int64)]),
    "apx_eam_forces": (C.c_int32, [_P, C.POINTER(Atoms), C.POINTER(NList), C.POINTER(EamParams), _P, _P, _P, _P]),
    "apx_ace_num_basis": (C.c_int64, [C.c_int32, C.c_int32]),
    "apx_ace_model_create": (C.c_int32, [_P, C.POINTER(AceDesc), C.POINTER(_P)]),
    "apx_ace_model_destroy": (None, [_P]),
    "apx_ace_model_set_coeffs": (C.c_int32, [_P, _P, _P, _P]),
    "apx_ace_energy_forces": (C.c_int32, [_P, C.POINTER(Atoms), C.POINTER(NList), _P, _P, _P, C.c_int64,
                                          C.c_int32, _P, _P, _P, _P]),
    "apx_blend": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "apx_blend_noalloc": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "apx_thermostat_energy_errors": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double,
                                                 C.c_double, _P]),
    "apx_thermostat_correct": (C.c_int32, [_P, C.POINTER(Atoms), _P, _P, C.POINTER(ThermoParams), C.c_int64,
                                           C.c_double, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "apx_md_create": (C.c_int32, [_P, C.POINTER(Atoms), C.POINTER(MdParams), C.POINTER(EamParams), _P,
                                  C.POINTER(PrecParams), C.POINTER(_P)]),
    "apx_md_destroy": (None, [_P]),
    "apx_md_init": (C.c_int32, [_P, _P, _P, _P]),
    "apx_verlet_step": (C.c_int32, [_P, _P, _P, _P, _P, C.c_int64, C.POINTER(MdStats)]),
    "apx_md_timings": (C.c_int32, [_P, C.POINTER(C.c_double)]),
    "apx_md_set_mlp": (C.c_int32, [_P, _P, C.c_double, C.c_double]),
    "apx_mlp_create": (C.c_int32, [_P, _P, _P, _P, C.POINTER(_P)]),
    "apx_mlp_destroy": (None, [_P]),
    "apx_mlp_get_params": (C.c_int32, [_P, _P, _P]),
    "apx_mlp_set_range": (C.c_int32, [_P, _P, _P]),
    "apx_features": (C.c_int32, [_P, C.POINTER(Atoms), C.POINTER(NList), _P, _P, _P, _P]),
    "apx_mlp_forward": (C.c_int32, [_P, _P, _P, C.c_int64, _P]),
    "apx_mlp_gradients": (C.c_int32, [_P, _P, _P, _P, _P, C.c_int64, _P, _P]),
    "apx_mlp_adam_step": (C.c_int32, [_P, _P, _P, C.c_float, C.c_float, C.c_float, C.c_float]),
    "apx_mlp_train_step": (C.c_int32, [_P, _P, _P, _P, _P, C.c_int64, C.c_float, _P]),
    "apx_mlp_infer_bf16": (C.c_int32, [_P, _P, _P, C.c_int64, _P]),
    "apx_mlp_precision": (C.c_int32, [_P, _P, _P, C.c_int64, C.c_double, C.c_double, _P, _P]),
    "apx_mlp_weight": (C.c_int32, [_P, _P, _P, _P, C.c_int64, C.c_double, C.c_double, _P]),
    "apx_mlp_labels": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P]),
    "apx_mlp_feature_stats": (C.c_int32, [_P, _P, C.c_int64, _P]),
    "apx_weighted_sum": (C.c_int32, [_P, C.c_int64, _P, _P, _P]),
}
MLP_PARAMS = 8705
APX_PREC_CSP_GIVEN = 1
APX_PREC_EXTRA_LOCAL = 2
WINDOW_PAST, WINDOW_CURRENT = 0, 1

_LIB = None


class ApxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"apx error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Loads libapx.so and declares its prototypes (raises if it is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2411_03002_amd.build_lib")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
