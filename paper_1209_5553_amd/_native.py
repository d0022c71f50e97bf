"""ctypes view of the C ABI declared in include/erem.h (argument marshalling only).

The shared library liberem.so is built in-tree by ``paper_1209_5553_amd.build``.
Loading fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liberem.so")

EREM_OK = 0
ERROR_NAMES = {
    -1: "EREM_EINVAL", -2: "EREM_ENOMEM", -3: "EREM_EDEVICE",
    -4: "EREM_ENOCONV", -5: "EREM_ENONFINITE",
}
METHOD_LEJA, METHOD_KRYLOV = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
LAW_CONSTANT, LAW_WATER = 0, 1


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("nx", c_int64), ("ny", c_int64), ("nz", c_int64),
                ("dx", c_double), ("dy", c_double), ("dz", c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("method", c_int32), ("precision", c_int32), ("tol_a", c_double),
                ("tol_r", c_double), ("p_order", c_int32), ("m_max", c_int32),
                ("max_substeps", c_int32), ("krylov_m", c_int32), ("chunk", c_int32),
                ("rho_max", c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("m_total", c_int32), ("substeps", c_int32), ("iterations", c_int32),
                ("restarts", c_int32), ("alpha", c_double), ("beta", c_double),
                ("est_err", c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelTimes(ctypes.Structure):
    _fields_ = [("leja_term_ms", c_double), ("leja_term_launches", c_int64),
                ("pcg_a_ms", c_double), ("pcg_a_launches", c_int64),
                ("pcg_b_ms", c_double), ("pcg_b_launches", c_int64),
                ("mg_ms", c_double), ("mg_cycles", c_int64),
                ("adj_rev_ms", c_double), ("adj_rev_launches", c_int64),
                ("bicg_ms", c_double), ("bicg_iterations", c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("terms_total", c_int64), ("terms_min", c_int32), ("terms_max", c_int32),
                ("failed", c_int32), ("tile_shape", c_int32), ("graph", c_int32),
                ("grid", c_int32), ("ms", c_double), ("leja_bytes", c_double), ("phases", c_int32),
                ("work_timed", c_int32), ("passes", c_int64), ("work_ms", c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


TAPE_MAX_SUBSTEPS = 256


class Tape(ctypes.Structure):
    _fields_ = [("substeps", c_int32), ("m", c_int32 * TAPE_MAX_SUBSTEPS),
                ("alpha", c_double), ("beta", c_double)]

    def as_dict(self):
        return {"substeps": self.substeps, "m": list(self.m[:self.substeps]),
                "alpha": self.alpha, "beta": self.beta}


_P = c_void_p           # device pointer / opaque handle
_PD = POINTER(c_double)  # host double array

# name -> (restype, argtypes); must cover every function of include/erem.h
SIGNATURES = {
    "erem_default_opts": (None, [POINTER(Opts)]),
    "erem_create": (c_int32, [POINTER(Grid), _P, POINTER(_P)]),
    "erem_destroy": (c_int32, [_P]),
    "erem_last_error": (c_char_p, [_P]),
    "erem_set_rock": (c_int32, [_P, _P, _P, c_double, c_double]),
    "erem_set_fluid": (c_int32, [_P, c_int32, c_double, c_double, c_double]),
    "erem_set_bc": (c_int32, [_P, c_double, c_double, c_double, c_double, c_int32]),
    "erem_assemble_transmissibilities": (c_int32, [_P, _P]),
    "erem_solve_pressure": (c_int32, [_P, c_double, c_int32, c_int32, _P, POINTER(Stats)]),
    "erem_set_face_fluxes": (c_int32, [_P, _P, _P, _P]),
    "erem_set_pressure_preconditioner": (c_int32, [_P, c_int32]),
    "erem_get_faces": (c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "erem_form_jacobian": (c_int32, [_P, _P]),
    "erem_get_jacobian": (c_int32, [_P, _P, _P]),
    "erem_set_jacobian": (c_int32, [_P, _P, _P]),
    "erem_phi1_apply": (c_int32, [_P, c_double, _P, _P, POINTER(Opts), POINTER(Stats)]),
    "erem_step": (c_int32, [_P, c_double, _P, POINTER(Opts), POINTER(Stats)]),
    "erem_step_frozen": (c_int32, [_P, c_double, _P, POINTER(Opts), POINTER(Stats)]),
    "erem_step_nonautonomous": (c_int32, [_P, c_double, c_double, c_double, c_double, c_double, _P,
                                          POINTER(Opts), POINTER(Stats)]),
    "erem_face_fluxes_from_pressure": (c_int32, [_P, _P]),
    "erem_step_pressure": (c_int32, [_P, c_double, _P, _P, c_double, c_double, POINTER(Opts), POINTER(Stats)]),
    "erem_shifted_solve": (c_int32, [_P, c_double, _P, _P, c_double, c_int32, POINTER(Stats)]),
    "erem_step_rosenbrock": (c_int32, [_P, c_double, c_int32, _P, c_double, POINTER(Stats)]),
    "erem_step_rosenbrock_nonautonomous": (c_int32, [_P, c_double, c_int32, _PD, _PD, c_double, c_double, _P,
                                                     c_double, POINTER(Stats)]),
    "erem_step_theta": (c_int32, [_P, c_double, c_double, _P, c_double, c_double, c_int32, POINTER(Stats)]),
    "erem_coupled_step": (c_int32, [_P, c_double, _P, c_double, POINTER(Opts), POINTER(Tape),
                                    POINTER(Tape), POINTER(Stats)]),
    "erem_coupled_step_adjoint": (c_int32, [_P, c_double, _P, c_double, POINTER(Opts), POINTER(Tape),
                                            c_int32, _P, _P, POINTER(Stats)]),
    "erem_batch_create": (c_int32, [c_int32, POINTER(Grid), _P, POINTER(_P)]),
    "erem_batch_destroy": (c_int32, [_P]),
    "erem_batch_last_error": (c_char_p, [_P]),
    "erem_batch_offsets": (c_int32, [_P, POINTER(c_int64)]),
    "erem_batch_set_problem": (c_int32, [_P, c_int32, _P, _P, c_double, c_double, c_double, c_double,
                                         c_double, c_double, c_double, c_double, c_double, _P]),
    "erem_batch_prepare": (c_int32, [_P, c_double, POINTER(Opts)]),
    "erem_batch_autotune": (c_int32, [_P, _P, c_int32, POINTER(c_int32)]),
    "erem_batch_run": (c_int32, [_P, _P, c_int32, c_int32, POINTER(BatchStats)]),
    "erem_batch_set_tile_shape": (c_int32, [_P, c_int32]),
    "erem_batch_profile": (c_int32, [_P, c_int32]),
    "erem_phi1_apply_noalloc": (c_int32, [POINTER(Grid), _P, c_double, _P, _P, POINTER(Opts), _P, POINTER(Stats)]),
    "erem_profile": (c_int32, [_P, c_int32]),
    "erem_profile_read": (c_int32, [_P, POINTER(KernelTimes)]),
    "erem_leja_points": (c_int32, [c_int32, _PD]),
    "erem_phi1_divided_differences": (c_int32, [c_double, c_double, _PD, c_int32, _PD]),
    "erem_phi2_divided_differences": (c_int32, [c_double, c_double, _PD, c_int32, _PD]),
}

_lib = None


def load():
    """Load liberem.so and attach the signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_1209_5553_amd.build` "
            "(the EREM path has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_opts() -> Opts:
    o = Opts()
    load().erem_default_opts(ctypes.byref(o))
    return o
