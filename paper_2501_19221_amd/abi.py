"""The C ABI of libqpa (include/qpa.h) as ctypes declarations: enums, structs and the
signature of every entry point.  No torch here, so that host-only tools (a sanitizer
build's checks) can load a library copy with `load(path)` alone; qpa.py loads the
product library through it after torch has brought up the HIP runtime."""
from __future__ import annotations

import ctypes

# ---- enums (mirror include/qpa.h) ---------------------------------------------------
QPA_OK, QPA_E_ARG, QPA_E_SHAPE, QPA_E_ASYM, QPA_E_RANGE, QPA_E_WORKSPACE, QPA_E_DEVICE, \
    QPA_E_UNSUPPORTED = range(8)
QPA_KIND_QUBO, QPA_KIND_ISING = 0, 1
QPA_FMT_DENSE, QPA_FMT_CSR = 0, 1
QPA_I8, QPA_I16, QPA_I32, QPA_F32 = 0, 1, 2, 3
QPA_PREC_FP32, QPA_PREC_BF16 = 0, 1
QPA_BATCH_SPARSE, QPA_BATCH_DENSE = 1, 2
QPA_PATH_ALL, QPA_PATH_DENSE_RESIDENT, QPA_PATH_DENSE_TILED, QPA_PATH_DENSE_MFMA, QPA_PATH_CSR, \
    QPA_PATH_BATCH_SPARSE, QPA_PATH_BATCH_DENSE, QPA_PATH_CSR_RESIDENT, QPA_PATH_SBM_DENSE, \
    QPA_PATH_SBM_CSR, QPA_PATH_SBM_CSR_RESIDENT, QPA_PATH_BATCH_DENSE_I8, \
    QPA_PATH_CSR_BINNED, QPA_PATH_BATCH_SPARSE_I8 = range(-1, 13)
QPA_SOLVE_STREAMED = 4
QPA_SOLVE_GRAPH = 8
QPA_SOLVE_BINNED = 16
QPA_TUNE_BINNED = -1
QPA_SPECTRUM_MAX_R = 4096
QPA_SPECTRUM_EXACT_ONLY = 1

EXPORTED = ["qpa_create", "qpa_destroy", "qpa_last_error", "qpa_status_string",
            "qpa_workspace_size", "qpa_solve", "qpa_steps", "qpa_energy", "qpa_version",
            "qpa_profile_enable", "qpa_profile_read", "qpa_workspace_size_batch",
            "qpa_solve_batch", "qpa_workspace_size_relaxed", "qpa_relaxed_grad",
            "qpa_profile_read_path", "qpa_batch_paths", "qpa_workspace_size_sbm",
            "qpa_sbm_solve", "qpa_sbm_steps", "qpa_spectral_radius",
            "qpa_workspace_size_spectrum", "qpa_spectrum", "qpa_autotune", "qpa_tune_set",
            "qpa_solve_noalloc", "qpa_workspace_size_relaxed_batch", "qpa_relaxed_grad_batch",
            "qpa_autotune_batch", "qpa_solve_track"]
QPA_NOALLOC_WORKSPACE_BYTES = 64 << 20
QPA_NOALLOC_MAX_STEPS = 65536


class qpa_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("kind", ctypes.c_int32), ("format", ctypes.c_int32),
                ("coupling_dtype", ctypes.c_int32), ("index_dtype", ctypes.c_int32),
                ("linear_dtype", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("dense", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("linear", ctypes.c_void_p)]


class qpa_params(ctypes.Structure):
    _fields_ = [("replicas", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("eta", ctypes.c_float), ("alpha", ctypes.c_float),
                ("lambda0", ctypes.c_float), ("sigma0", ctypes.c_float),
                ("lambda_table", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]


class qpa_outputs(ctypes.Structure):
    _fields_ = [("spins", ctypes.c_void_p), ("energy", ctypes.c_void_p),
                ("energy_i64", ctypes.c_void_p), ("best", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("m", ctypes.c_void_p)]


class qpa_track_outputs(ctypes.Structure):
    _fields_ = [("best_energy", ctypes.c_void_p), ("best_step", ctypes.c_void_p),
                ("best_spins", ctypes.c_void_p)]


class qpa_sbm_params(ctypes.Structure):
    _fields_ = [("replicas", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("a0", ctypes.c_float), ("c0", ctypes.c_float), ("dt", ctypes.c_float),
                ("sigma0", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("power_iters", ctypes.c_int32), ("flags", ctypes.c_int32)]


_P = ctypes.c_void_p
_S = ctypes.c_int
_sig = {
    "qpa_create": (_S, [ctypes.POINTER(_P), ctypes.c_int]),
    "qpa_destroy": (None, [_P]),
    "qpa_last_error": (ctypes.c_char_p, [_P]),
    "qpa_status_string": (ctypes.c_char_p, [_S]),
    "qpa_version": (ctypes.c_char_p, []),
    "qpa_workspace_size": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params),
                                ctypes.POINTER(ctypes.c_size_t)]),
    "qpa_solve": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params), _P,
                       ctypes.c_size_t, _P, ctypes.POINTER(qpa_outputs)]),
    "qpa_solve_noalloc": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params), _P,
                               ctypes.POINTER(qpa_outputs)]),
    "qpa_solve_track": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params),
                             ctypes.c_int32, _P, ctypes.c_size_t, _P, ctypes.POINTER(qpa_outputs),
                             ctypes.POINTER(qpa_track_outputs)]),
    "qpa_steps": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params),
                       ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "qpa_energy": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params), _P, _P,
                        _P, _P, _P, ctypes.c_size_t, _P]),
    "qpa_workspace_size_batch": (_S, [_P, ctypes.c_int32, ctypes.POINTER(qpa_problem),
                                      ctypes.POINTER(qpa_params),
                                      ctypes.POINTER(ctypes.c_size_t)]),
    "qpa_solve_batch": (_S, [_P, ctypes.c_int32, ctypes.POINTER(qpa_problem),
                             ctypes.POINTER(qpa_params), _P, ctypes.c_size_t, _P,
                             ctypes.POINTER(qpa_outputs)]),
    "qpa_workspace_size_relaxed": (_S, [_P, ctypes.POINTER(qpa_problem),
                                        ctypes.POINTER(qpa_params), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "qpa_relaxed_grad": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params),
                              ctypes.c_int32, ctypes.c_double, _P, ctypes.c_size_t, _P, _P, _P,
                              _P, _P]),
    "qpa_workspace_size_relaxed_batch": (_S, [_P, ctypes.c_int32, ctypes.POINTER(qpa_problem),
                                              ctypes.POINTER(qpa_params), ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "qpa_relaxed_grad_batch": (_S, [_P, ctypes.c_int32, ctypes.POINTER(qpa_problem),
                                    ctypes.POINTER(qpa_params), ctypes.c_int32, ctypes.c_double,
                                    _P, ctypes.c_size_t, _P, _P, _P, _P, _P]),
    "qpa_profile_enable": (_S, [_P, ctypes.c_int32]),
    "qpa_profile_read": (_S, [_P, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "qpa_profile_read_path": (_S, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "qpa_batch_paths": (_S, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "qpa_workspace_size_sbm": (_S, [_P, ctypes.POINTER(qpa_problem),
                                    ctypes.POINTER(qpa_sbm_params),
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "qpa_sbm_solve": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_sbm_params), _P,
                           ctypes.c_size_t, _P, ctypes.POINTER(qpa_outputs)]),
    "qpa_sbm_steps": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_sbm_params),
                           ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_size_t,
                           _P]),
    "qpa_spectral_radius": (_S, [_P, ctypes.POINTER(qpa_problem),
                                 ctypes.POINTER(qpa_sbm_params), _P, ctypes.c_size_t, _P, _P]),
    "qpa_autotune": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params),
                          ctypes.c_int32, _P, ctypes.c_size_t, _P,
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "qpa_tune_set": (_S, [_P, ctypes.POINTER(qpa_problem), ctypes.POINTER(qpa_params),
                          ctypes.c_int32]),
    "qpa_autotune_batch": (_S, [_P, ctypes.c_int32, ctypes.POINTER(qpa_problem),
                                ctypes.POINTER(qpa_params), ctypes.c_int32, _P,
                                ctypes.POINTER(ctypes.c_double)]),
    "qpa_workspace_size_spectrum": (_S, [_P, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "qpa_spectrum": (_S, [_P, ctypes.c_int64, ctypes.c_int32, _P, _P, ctypes.c_int32,
                          ctypes.c_int32, _P, ctypes.c_size_t, _P, _P, _P, _P, _P, _P]),
}


def load(path: str) -> ctypes.CDLL:
    """Load a build of libqpa and give every entry point its signature."""
    lib = ctypes.CDLL(path)
    for name, (res, args) in _sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib
