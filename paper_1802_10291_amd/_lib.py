"""ctypes binding of libmci (include/mci.h): argument marshalling only.

The shared library must have been built (``__graft_entry__.build()`` or
``python -m paper_1802_10291_amd.build``); there is no fallback of any kind, and a
missing library raises at import of the first call.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmci.so")

MCI_MAX_CHANNELS = 4
MCI_MAX_OPS = 4
MCI_N1_DEFAULT = -(2**63)
MCI_ALLOW_SINGULAR_ZERO = 1

MCI_MULT_DERIV, MCI_MULT_HILBERT, MCI_MULT_TABLE = 0, 1, 2
MCI_OUT_IDENTITY, MCI_OUT_HILBERT, MCI_OUT_DERIV = 0, 1, 2
MCI_F32, MCI_F64 = 0, 1
MCI_STORE_NATIVE, MCI_STORE_F16 = 0, 1

STATUS = {0: "MCI_OK", 1: "MCI_E_INVALID_ARG", 2: "MCI_E_SINGULAR", 3: "MCI_E_ILL_CONDITIONED",
          4: "MCI_E_UNSUPPORTED", 5: "MCI_E_OUT_OF_MEMORY", 6: "MCI_E_DEVICE"}


class mci_channel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32), ("table", ctypes.POINTER(ctypes.c_double))]


class mci_plan_desc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("n_ops", ctypes.c_int32),
        ("N", ctypes.c_int64), ("n1", ctypes.c_int64), ("n_out", ctypes.c_int64),
        ("ch", mci_channel * MCI_MAX_CHANNELS),
        ("ops", ctypes.c_int32 * MCI_MAX_OPS), ("op_orders", ctypes.c_int32 * MCI_MAX_OPS),
        ("real_io", ctypes.c_int32), ("precision", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("cond_max", ctypes.c_double),
    ]


class mci_plan_info_t(ctypes.Structure):
    _fields_ = [("max_cond", ctypes.c_double), ("n_singular", ctypes.c_int64), ("first_singular", ctypes.c_int64),
                ("n1", ctypes.c_int64), ("fft_len_fwd", ctypes.c_int64), ("fft_len_inv", ctypes.c_int64),
                ("path", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mci_plan2d_desc(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32), ("scale", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("storage", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# every symbol the header declares
EXPORTS = ["mci_plan", "mci_plan_destroy", "mci_plan_info", "mci_workspace_size", "mci_reconstruct_1d",
           "mci_plan_2d", "mci_upsample_2d", "mci_status_string", "mci_last_error"]

_lib = None


class MCIError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} {detail}".strip())


def load(path: str = LIB_PATH):
    """Load libmci.so and declare its signatures (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with __graft_entry__.build() "
                          "(python -m paper_1802_10291_amd.build); there is no fallback")
    # PyTorch ships its own HIP runtime under the same soname as the system one: loading
    # torch first makes libmci bind to that runtime, so both share one device context and
    # torch's stream handles are valid here.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    lib.mci_plan.argtypes = [P(mci_plan_desc), i32, P(vp)]
    lib.mci_plan_destroy.argtypes = [vp]
    lib.mci_plan_info.argtypes = [vp, P(mci_plan_info_t)]
    lib.mci_workspace_size.argtypes = [vp, i64, P(sz)]
    lib.mci_reconstruct_1d.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    lib.mci_plan_2d.argtypes = [P(mci_plan2d_desc), i32, P(vp)]
    lib.mci_upsample_2d.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    lib.mci_status_string.argtypes = [i32]
    lib.mci_status_string.restype = ctypes.c_char_p
    lib.mci_last_error.argtypes = []
    lib.mci_last_error.restype = ctypes.c_char_p
    for name in ("mci_plan", "mci_plan_destroy", "mci_plan_info", "mci_workspace_size", "mci_reconstruct_1d",
                 "mci_plan_2d", "mci_upsample_2d"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != 0:
        detail = load().mci_last_error().decode(errors="replace")
        raise MCIError(status, where, detail)


# ----------------------------------------------------------------------------- raw calls
def mci_plan(desc: mci_plan_desc, device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().mci_plan(ctypes.byref(desc), device, ctypes.byref(h)), "mci_plan")
    return h.value


def mci_plan_destroy(plan: int) -> None:
    check(load().mci_plan_destroy(plan), "mci_plan_destroy")


def mci_plan_info(plan: int) -> mci_plan_info_t:
    info = mci_plan_info_t()
    check(load().mci_plan_info(plan, ctypes.byref(info)), "mci_plan_info")
    return info


def mci_workspace_size(plan: int, batch: int) -> int:
    n = ctypes.c_size_t()
    check(load().mci_workspace_size(plan, batch, ctypes.byref(n)), "mci_workspace_size")
    return n.value


def mci_reconstruct_1d(plan: int, g_ptr: int, y_ptr: int, batch: int, ws_ptr: int, ws_bytes: int,
                       stream: int) -> None:
    check(load().mci_reconstruct_1d(plan, g_ptr, y_ptr, batch, ws_ptr, ws_bytes, stream), "mci_reconstruct_1d")


def mci_plan_2d(desc: mci_plan2d_desc, device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().mci_plan_2d(ctypes.byref(desc), device, ctypes.byref(h)), "mci_plan_2d")
    return h.value


def mci_upsample_2d(plan: int, lr_ptr: int, hr_ptr: int, batch: int, ws_ptr: int, ws_bytes: int,
                    stream: int) -> None:
    check(load().mci_upsample_2d(plan, lr_ptr, hr_ptr, batch, ws_ptr, ws_bytes, stream), "mci_upsample_2d")


# ----------------------------------------------------------------------------- refiner
REFINER_EXPORTS = ["mci_refiner_create", "mci_refiner_destroy", "mci_refiner_num_params", "mci_refiner_get_params",
                   "mci_refiner_set_params", "mci_refiner_get_grads", "mci_refiner_workspace_size",
                   "mci_refiner_forward", "mci_refiner_backward", "mci_refiner_train_step", "mci_refiner_last_error"]
EXPORTS += REFINER_EXPORTS


def load_refiner():
    lib = load()
    if getattr(lib, "_refiner_ready", False):
        return lib
    vp, i64, i32, sz, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t, ctypes.c_float
    P = ctypes.POINTER
    lib.mci_refiner_create.argtypes = [i32, ctypes.c_uint64, P(vp)]
    lib.mci_refiner_destroy.argtypes = [vp]
    lib.mci_refiner_num_params.argtypes = []
    lib.mci_refiner_num_params.restype = i64
    lib.mci_refiner_get_params.argtypes = [vp, P(f32), P(f32)]
    lib.mci_refiner_set_params.argtypes = [vp, P(f32), f32]
    lib.mci_refiner_get_grads.argtypes = [vp, P(f32)]
    lib.mci_refiner_workspace_size.argtypes = [i64, i32, i32, P(sz)]
    lib.mci_refiner_forward.argtypes = [vp, vp, vp, i64, i32, i32, i32, vp, vp, vp, sz, vp]
    lib.mci_refiner_backward.argtypes = [vp, vp, vp, i64, i32, i32, vp, P(i32), vp, sz, vp]
    lib.mci_refiner_train_step.argtypes = [vp, vp, vp, i64, i32, i32, f32, vp, P(i32), vp, sz, vp]
    lib.mci_refiner_last_error.argtypes = []
    lib.mci_refiner_last_error.restype = ctypes.c_char_p
    for n in ("mci_refiner_create", "mci_refiner_destroy", "mci_refiner_get_params", "mci_refiner_set_params",
              "mci_refiner_get_grads", "mci_refiner_workspace_size", "mci_refiner_forward", "mci_refiner_backward",
              "mci_refiner_train_step"):
        getattr(lib, n).restype = i32
    lib._refiner_ready = True
    return lib


def rcheck(status: int, where: str):
    if status != 0:
        raise MCIError(status, where, load_refiner().mci_refiner_last_error().decode(errors="replace"))
