"""ctypes declarations of the C ABI in include/abc_dtn.h (argument marshalling
only; every computation happens in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# ABC_DTN_LIBRARY names another build of the same ABI (the host-sanitizer one)
LIB_PATH = os.environ.get("ABC_DTN_LIBRARY") or os.path.join(HERE, "libabc_dtn.so")

ABC_OK, ABC_EINVAL, ABC_ENOMEM, ABC_EDEVICE, ABC_EUNSTABLE, ABC_ENOTSUP, ABC_EIO = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "ABC_OK", -1: "ABC_EINVAL", -2: "ABC_ENOMEM", -3: "ABC_EDEVICE",
                -4: "ABC_EUNSTABLE", -5: "ABC_ENOTSUP", -6: "ABC_EIO"}
ABC_BATCH_GRAPH = 1
ABC_FLAG_NONFINITE, ABC_FLAG_W_INCREASE = 1, 2
ORDERS = {"dirichlet": 0, "periodic": 1, "zeroth": 2, "first": 3, "second": 4}
FORMS = {"box": 0, "faces": 1}
DTYPES = {"c128": 0, "c64": 1}
PATHS = {"auto": 0, "staged": 1, "fused": 2, "onepass": 3}
OBJECTIVES = {"prob": 0, "energy": 1}

EXPORTED = ["abc_params_default", "abc_setup", "abc_step", "abc_diagnostics", "abc_aux_elems",
            "abc_export", "abc_path", "abc_device_bytes", "abc_last_error", "abc_destroy",
            "abc_step_timed", "abc_launch_label", "abc_adjoint", "abc_tune", "abc_setup_batch",
            "abc_step_batch", "abc_tune_batch", "abc_batch_aux_elems", "abc_batch_launch_groups",
            "abc_batch_tile_depth", "abc_destroy_batch", "abc_h2_objective",
            "abc_effective_potential", "abc_potential_iterations", "abc_potential_unconverged", "abc_state_save",
            "abc_state_load",
            "abc_diagnostics_noalloc", "abc_step_monitored"]


class AbcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("radius", ctypes.c_int), ("order", ctypes.c_int), ("form", ctypes.c_int),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("s2", ctypes.c_double),
        ("window", ctypes.c_int), ("fejer", ctypes.c_int), ("dtype", ctypes.c_int),
        ("batch", ctypes.c_int), ("meanfield", ctypes.c_int),
        ("t0", ctypes.c_double), ("t3", ctypes.c_double),
        ("path", ctypes.c_int), ("diag_every", ctypes.c_int), ("reserved", ctypes.c_int * 2),
        ("s3", ctypes.c_double), ("s4", ctypes.c_double),
        ("v0", ctypes.c_double), ("a_yukawa", ctypes.c_double), ("e2", ctypes.c_double),
        ("pcg_tol", ctypes.c_double), ("pcg_maxit", ctypes.c_int), ("pcg_fixed", ctypes.c_int),
        ("reserved2", ctypes.c_int * 2),
    ]


class AbcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libabc_dtn.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(AbcParams)
    vp = ctypes.c_void_p
    lib.abc_params_default.argtypes = [P]
    lib.abc_params_default.restype = None
    lib.abc_setup.argtypes = [P, ctypes.POINTER(vp)]
    lib.abc_setup.restype = ctypes.c_int
    lib.abc_step.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp]
    lib.abc_step.restype = ctypes.c_int
    lib.abc_step_timed.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, vp, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.abc_step_timed.restype = ctypes.c_int
    lib.abc_launch_label.argtypes = [vp, ctypes.c_int]
    lib.abc_launch_label.restype = ctypes.c_char_p
    lib.abc_adjoint.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp,
                                ctypes.POINTER(ctypes.c_double), vp]
    lib.abc_adjoint.restype = ctypes.c_int
    lib.abc_tune.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int)]
    lib.abc_tune.restype = ctypes.c_int
    lib.abc_setup_batch.argtypes = [P, ctypes.c_int, ctypes.POINTER(vp)]
    lib.abc_setup_batch.restype = ctypes.c_int
    lib.abc_step_batch.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    lib.abc_step_batch.restype = ctypes.c_int
    lib.abc_tune_batch.argtypes = [vp, vp, vp, vp, vp]
    lib.abc_tune_batch.restype = ctypes.c_int
    lib.abc_batch_aux_elems.argtypes = [vp, ctypes.c_int]
    lib.abc_batch_aux_elems.restype = ctypes.c_size_t
    lib.abc_batch_launch_groups.argtypes = [vp]
    lib.abc_batch_launch_groups.restype = ctypes.c_int
    lib.abc_batch_tile_depth.argtypes = [vp, ctypes.c_int]
    lib.abc_batch_tile_depth.restype = ctypes.c_int
    lib.abc_destroy_batch.argtypes = [vp]
    lib.abc_destroy_batch.restype = None
    lib.abc_h2_objective.argtypes = [P, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.abc_h2_objective.restype = ctypes.c_int
    lib.abc_effective_potential.argtypes = [vp, vp, vp, vp, vp]
    lib.abc_effective_potential.restype = ctypes.c_int
    lib.abc_potential_iterations.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    lib.abc_potential_iterations.restype = ctypes.c_int
    lib.abc_potential_unconverged.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    lib.abc_potential_unconverged.restype = ctypes.c_int
    lib.abc_state_save.argtypes = [vp, vp, vp, ctypes.c_longlong, ctypes.c_char_p, vp]
    lib.abc_state_save.restype = ctypes.c_int
    lib.abc_state_load.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_longlong), ctypes.c_char_p, vp]
    lib.abc_state_load.restype = ctypes.c_int
    lib.abc_diagnostics.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.abc_diagnostics.restype = ctypes.c_int
    lib.abc_diagnostics_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.abc_diagnostics_noalloc.restype = ctypes.c_int
    lib.abc_step_monitored.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    lib.abc_step_monitored.restype = ctypes.c_int
    lib.abc_aux_elems.argtypes = [vp]
    lib.abc_aux_elems.restype = ctypes.c_size_t
    lib.abc_export.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t]
    lib.abc_export.restype = ctypes.c_int
    lib.abc_path.argtypes = [vp]
    lib.abc_path.restype = ctypes.c_int
    lib.abc_device_bytes.argtypes = [vp]
    lib.abc_device_bytes.restype = ctypes.c_size_t
    lib.abc_last_error.argtypes = []
    lib.abc_last_error.restype = ctypes.c_char_p
    lib.abc_destroy.argtypes = [vp]
    lib.abc_destroy.restype = None
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != ABC_OK:
        msg = load().abc_last_error().decode(errors="replace")
        raise AbcError(status, msg)
