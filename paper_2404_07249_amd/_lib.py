"""ctypes declarations for libpb3.so (the C ABI in include/pb3.h)."""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PB3_LIBRARY names another build of the same library (the sanitizer build)
LIB_PATH = os.environ.get("PB3_LIBRARY") or os.path.join(_HERE, "libpb3.so")

PB3_OK = 0
PB3_EINVAL, PB3_ENOMEM, PB3_EDEVICE, PB3_EUNSUPPORTED = 1, 2, 3, 4
STATUS = {0: "PB3_OK", 1: "PB3_EINVAL", 2: "PB3_ENOMEM", 3: "PB3_EDEVICE", 4: "PB3_EUNSUPPORTED", 5: "PB3_EBUSY"}

FLAG_EDGES_HMPC = 0x1
FLAG_HOST_ONLY = 0x2
FLAG_FULL_GRID = 0x4
FLAG_STRICT = 0x8
FLAG_EXT_WORKSPACE = 0x10
FLAG_STAGE_TIMING = 0x20
FLAG_NO_FUSION = 0x40
FLAG_AUTOTUNE = 0x80
FLAG_POWER_ONLY = 0x100
FLAG_LMAX2 = 0x200
FLAG_LMAX4 = 0x400
FLAG_BK_FISHER = 0x800
BATCH_GRAPH = 0x1
WINDOW_SCRATCH = 514
BATCH_EXT_WORKSPACE = 0x2

PREC_FP32 = 0
PREC_MIXED_BF16X3 = 1

# every symbol include/pb3.h declares: (name, restype, argtypes)
SIGNATURES = [
    ("pb3_plan_create", C.c_int,
     [C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int, C.c_uint, C.POINTER(C.c_void_p)]),
    ("pb3_plan_destroy", C.c_int, [C.c_void_p]),
    ("pb3_plan_workspace_bytes", C.c_size_t, [C.c_void_p]),
    ("pb3_plan_bind_workspace", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("pb3_n_bins", C.c_int, [C.c_void_p]),
    ("pb3_n_triplets", C.c_int, [C.c_void_p]),
    ("pb3_grid", C.c_int, [C.c_void_p]),
    ("pb3_contract_grid", C.c_int, [C.c_void_p]),
    ("pb3_grid3", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_plan_launch_shape", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_get_bins", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_get_triplets", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pb3_norm", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_power", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_bispectrum", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("pb3_polyspectra", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("pb3_window_normalize", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_masked_power_workspace_bytes", C.c_size_t, [C.c_void_p]),
    ("pb3_bispectrum_linear_workspace_bytes", C.c_size_t, [C.c_void_p, C.c_int]),
    ("pb3_bispectrum_linear", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("pb3_masked_power", C.c_int,
     [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_size_t, C.c_void_p]),
    ("pb3_n_ell", C.c_int, [C.c_void_p]),
    ("pb3_multipole_mixing", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("pb3_weights_table_len", C.c_int, [C.c_void_p]),
    ("pb3_plan_set_weights", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_double]),
    ("pb3_multipoles_workspace_bytes", C.c_size_t, [C.c_void_p]),
    ("pb3_multipoles", C.c_int,
     [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("pb3_stage_times", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)]),
    ("pb3_stage_timing_reset", C.c_int, [C.c_void_p]),
    ("pb3_stage_name", C.c_char_p, [C.c_int]),
    ("pb3_batch_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_uint, C.POINTER(C.c_void_p)]),
    ("pb3_batch_destroy", C.c_int, [C.c_void_p]),
    ("pb3_batch_workspace_bytes", C.c_size_t, [C.c_void_p]),
    ("pb3_batch_bind_workspace", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("pb3_batch_run", C.c_int,
     [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    ("pb3_batch_launches", C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    ("pb3_batch_groups", C.c_int, [C.c_void_p]),
    ("pb3_bispectrum_batched", C.c_int,
     [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_void_p]),
    ("pb3_power_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pb3_status_string", C.c_char_p, [C.c_int]),
    ("pb3_last_error", C.c_char_p, []),
]

_lib = None


class Pb3Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libpb3.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} not found: build the HIP library first (python -m paper_2404_07249_amd.build); "
            "there is no CPU fallback"
        )
    # torch first: the library then binds to the HIP runtime torch already
    # loaded, so both share one runtime (device memory and streams pass
    # between them); loading the library first would let torch find a
    # second, mismatched runtime and fail to initialise the GPU.
    import torch  # noqa: F401

    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != PB3_OK:
        msg = load().pb3_last_error().decode(errors="replace")
        raise Pb3Error(status, msg)
