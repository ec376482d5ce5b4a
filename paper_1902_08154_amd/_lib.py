"""ctypes declarations of libqp_pt2.so (include/qp_pt2.h).  Loading fails loudly
when the library has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqp_pt2.so")

QP_OK = 0
QP_E_ARG = -1
QP_E_NORB = -2
QP_E_ELEC = -3
QP_E_DUP = -4
QP_E_NOINT = -5
QP_E_OOM = -6
QP_E_HIP = -7
QP_E_STATES = -8
QP_E_OVERFLOW = -9
QP_E_NOCONV = -10

QP_FLAG_FINGERPRINT = 1
QP_FLAG_NOCHECK = 2
QP_FLAG_REUSE_INTEGRALS = 4
QP_NOALLOC_MAX_DET = 1 << 18
QP_SPLIT_NEVER = 0
QP_SPLIT_AUTO = 1
QP_SPLIT_ALWAYS = 2
QP_PROBE_F64_FMA = 0
QP_PROBE_I32_ADD = 1
QP_PROBE_MIXED = 2
QP_SIGMA_S2 = 8
QP_SIGMA_REUSE = 16
QP_MAX_STATES = 4
QP_MAX_SYSTEMS = 4096

ERROR_NAMES = {
    QP_E_ARG: "QP_E_ARG", QP_E_NORB: "QP_E_NORB", QP_E_ELEC: "QP_E_ELEC", QP_E_DUP: "QP_E_DUP",
    QP_E_NOINT: "QP_E_NOINT", QP_E_OOM: "QP_E_OOM", QP_E_HIP: "QP_E_HIP", QP_E_STATES: "QP_E_STATES",
    QP_E_OVERFLOW: "QP_E_OVERFLOW", QP_E_NOCONV: "QP_E_NOCONV",
}


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_alpha", ctypes.c_uint64),
        ("n_cells", ctypes.c_uint64),
        ("fingerprint", ctypes.c_uint64),
        ("n_coarse", ctypes.c_uint64),
        ("n_candidates", ctypes.c_uint64),
        ("overflow", ctypes.c_uint64),
        ("n_connections", ctypes.c_uint64),
        ("n_alpha_general", ctypes.c_uint64),
        ("S", ctypes.c_double * QP_MAX_STATES),
        ("min_abs_delta", ctypes.c_double),
        ("Z", ctypes.c_double * QP_MAX_STATES),
        ("e_rpt2", ctypes.c_double * QP_MAX_STATES),
        ("n_fine", ctypes.c_uint64),
        ("n_alpha_clean", ctypes.c_uint64),
    ]


class System(ctypes.Structure):
    """qp_system of include/qp_pt2.h (device pointers as integers)."""
    _fields_ = [
        ("n_orb", ctypes.c_int),
        ("n_states", ctypes.c_int),
        ("n_det", ctypes.c_int64),
        ("h", ctypes.c_void_p),
        ("eri_packed", ctypes.c_void_p),
        ("dets", ctypes.c_void_p),
        ("coefs", ctypes.c_void_p),
        ("E0", ctypes.c_void_p),
        ("n_select", ctypes.c_int64),
        ("e_pt2", ctypes.c_void_p),
        ("sel_dets", ctypes.c_void_p),
        ("sel_e", ctypes.c_void_p),
        ("n_sel", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
        ("eps_gen", ctypes.c_void_p),
        ("grad_e_pt2", ctypes.c_void_p),
        ("grad_coefs", ctypes.c_void_p),
        ("grad_E0", ctypes.c_void_p),
        ("grad_h", ctypes.c_void_p),
    ]


# every entry point declared in include/qp_pt2.h
EXPORTS = ("qp_create", "qp_destroy", "qp_last_error", "qp_set_integrals", "qp_pt2",
           "qp_pt2_backward", "qp_generator_order", "qp_pt2_generators", "qp_pt2_stochastic",
           "qp_pt2_batched", "qp_sigma", "qp_davidson", "qp_energy", "qp_set_timing", "qp_last_timing",
           "qp_set_split", "qp_generator_order_noalloc", "qp_alu_probe")

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1902_08154_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.qp_create.argtypes = [ctypes.POINTER(_P), _I]
    lib.qp_create.restype = _I
    lib.qp_destroy.argtypes = [_P]
    lib.qp_destroy.restype = None
    lib.qp_last_error.argtypes = [_P]
    lib.qp_last_error.restype = ctypes.c_char_p
    lib.qp_set_integrals.argtypes = [_P, _P, _P, _I, _P]
    lib.qp_set_integrals.restype = _I
    lib.qp_pt2.argtypes = [_P, _P, _P, _I64, _I, _P, _I64, _I, _P, _P, _P, _P, _P, _P, _P]
    lib.qp_pt2.restype = _I
    lib.qp_pt2_backward.argtypes = [_P, _P, _P, _I64, _I, _P, _P, _I, _P, _P, _P, _P, _P]
    lib.qp_pt2_backward.restype = _I
    lib.qp_generator_order.argtypes = [_P, _P, _P, _I64, _I, _I, _P, _P]
    lib.qp_generator_order.restype = _I
    lib.qp_generator_order_noalloc.argtypes = [_P, _P, _P, _I64, _I, _I, _P, _P]
    lib.qp_generator_order_noalloc.restype = _I
    lib.qp_pt2_generators.argtypes = [_P, _P, _P, _I64, _I, _P, _P, _I64, _I64, _I, _P, _P, _P, _P, _P, _P]
    lib.qp_pt2_generators.restype = _I
    lib.qp_pt2_stochastic.argtypes = [_P, _P, _P, _I64, _I, _P, _P, _I64, ctypes.c_double, _I64, _I64, _I64, _I,
                                      _P, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.qp_pt2_stochastic.restype = _I
    lib.qp_pt2_batched.argtypes = [_P, _I, ctypes.POINTER(System), _I, _I, _P]
    lib.qp_pt2_batched.restype = _I
    lib.qp_sigma.argtypes = [_P, _P, _I64, _I, _P, _I, _P, _P]
    lib.qp_sigma.restype = _I
    lib.qp_davidson.argtypes = [_P, _P, _I64, _I, _P, ctypes.c_double, _I, _I, _P, _P, _P, _P, _P]
    lib.qp_davidson.restype = _I
    lib.qp_energy.argtypes = [_P, _P, _P, _I64, _I, _I, _P, _P]
    lib.qp_energy.restype = _I
    lib.qp_set_timing.argtypes = [_P, _I]
    lib.qp_set_timing.restype = _I
    lib.qp_last_timing.argtypes = [_P, ctypes.POINTER(ctypes.c_double)]
    lib.qp_last_timing.restype = _I
    lib.qp_set_split.argtypes = [_P, _I]
    lib.qp_set_split.restype = _I
    lib.qp_alu_probe.argtypes = [_P, _I, _I64, _P, ctypes.POINTER(ctypes.c_double)]
    lib.qp_alu_probe.restype = _I
    _lib = lib
    return lib
