"""ctypes binding of libaahrt.so (argument marshalling only; every step runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libaahrt.so')

AAHRT_OK = 0
AAHRT_E_INVALID = -1
AAHRT_E_HIP = -2
AAHRT_E_NOMEM = -3
AAHRT_E_UNSUPPORTED = -4

SOLVE_FISTA = 0
SOLVE_ISTA = 1
SOLVE_NO_GRAPH = 2

EXPORTED = ['aahrt_version', 'aahrt_last_error', 'aahrt_plan_create', 'aahrt_plan_destroy',
            'aahrt_plan_query', 'aahrt_forward', 'aahrt_adjoint', 'aahrt_lambda_max',
            'aahrt_operator_norm2', 'aahrt_sparse_solve', 'aahrt_velocity', 'aahrt_set_wavelet',
            'aahrt_adjoint_direct', 'aahrt_adjoint_grid',
            'aahrt_profile_enable', 'aahrt_profile_read', 'aahrt_adjoint_noalloc']

KERNELS = ['model_r2c', 'nufft_interp', 'data_c2r', 'data_r2c', 'nufft_spread', 'model_c2r',
           'residual_r2c', 'model_c2r_update', 'model_update_r2c']


class Params(ctypes.Structure):
    _fields_ = [('nt', ctypes.c_int32), ('dt', ctypes.c_double),
                ('ntau', ctypes.c_int32), ('dtau', ctypes.c_double),
                ('nq', ctypes.c_int32), ('q_min', ctypes.c_double), ('q_max', ctypes.c_double),
                ('ntheta', ctypes.c_int32), ('stretch', ctypes.c_int32), ('nfft', ctypes.c_int32),
                ('nufft_tol', ctypes.c_double), ('sigma', ctypes.c_double),
                ('kernel_width', ctypes.c_int32), ('freq_tile', ctypes.c_int32),
                ('grid_dtype', ctypes.c_int32), ('gfst_kind', ctypes.c_int32),
                ('block_threads', ctypes.c_int32), ('freq_tile_adjoint', ctypes.c_int32),
                ('block_threads_adjoint', ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [('batch', ctypes.c_int32), ('ntraces', ctypes.c_int64),
                ('nt_stretch', ctypes.c_int32), ('dt_stretch', ctypes.c_double),
                ('nfft', ctypes.c_int32), ('nfreq', ctypes.c_int32), ('grid_size', ctypes.c_int32),
                ('kernel_width', ctypes.c_int32), ('sigma', ctypes.c_double), ('beta', ctypes.c_double),
                ('freq_tile', ctypes.c_int32), ('workspace_bytes', ctypes.c_int64),
                ('q_alias_ok', ctypes.c_int32), ('autotune_candidates', ctypes.c_int32),
                ('autotune_seconds', ctypes.c_double), ('freq_tile_adjoint', ctypes.c_int32),
                ('gfst_resident', ctypes.c_int32), ('nufft_error_estimate', ctypes.c_double),
                ('block_threads', ctypes.c_int32), ('block_threads_adjoint', ctypes.c_int32)]


class AahrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'aahrt error {code}: {msg}')
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f'{LIB_PATH} is missing: build it with paper_2505_00387_amd.build.build()')
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.aahrt_version.restype = ctypes.c_char_p
    lib.aahrt_last_error.restype = ctypes.c_char_p
    lib.aahrt_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Params), ctypes.c_int32,
                                      P, P, P, ctypes.c_int32]
    lib.aahrt_plan_destroy.argtypes = [P]
    lib.aahrt_plan_query.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.aahrt_forward.argtypes = [P, P, P, P]
    lib.aahrt_adjoint.argtypes = [P, P, P, P]
    lib.aahrt_adjoint_noalloc.argtypes = [P, P, P, P]
    lib.aahrt_lambda_max.argtypes = [P, P, P, P]
    lib.aahrt_operator_norm2.argtypes = [P, ctypes.c_int32, P, P]
    lib.aahrt_velocity.argtypes = [P, P, P, P, P]
    lib.aahrt_set_wavelet.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32]
    lib.aahrt_adjoint_direct.argtypes = [P, P, P, P]
    lib.aahrt_adjoint_grid.argtypes = [P, P, P, P]
    lib.aahrt_sparse_solve.argtypes = [P, P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, P]
    lib.aahrt_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.aahrt_profile_read.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTED[2:]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(code: int):
    if code != AAHRT_OK:
        raise AahrtError(code, load().aahrt_last_error().decode())
