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
                ("path", ctypes.c_int32), ("variant", ctypes.c_int32)]


class mci_plan2d_desc(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32), ("scale", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("storage", ctypes.c_int32), ("channels", ctypes.c_int32)]


MCI_VARIANT_MULTIPASS_R8, MCI_VARIANT_MULTIPASS_R4, MCI_VARIANT_FUSED_T1, MCI_VARIANT_FUSED_T2, \
    MCI_VARIANT_LINE_PASS, MCI_VARIANT_TWO_PASS, MCI_VARIANT_REAL_TWO_PASS = range(7)
MCI_NUM_VARIANTS = 7
VARIANT_NAMES = ["multipass_r8", "multipass_r4", "fused_t1", "fused_t2", "line_pass", "two_pass", "real_two_pass"]


class mci_tune_result(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("batch", ctypes.c_int64),
                ("ms", ctypes.c_double * MCI_NUM_VARIANTS)]


class mci_batch_item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("in_off", ctypes.c_int64), ("out_off", ctypes.c_int64)]


# every symbol the header declares
EXPORTS = ["mci_plan", "mci_plan_destroy", "mci_plan_info", "mci_plan_kernel_name", "mci_workspace_size", "mci_reconstruct_1d",
           "mci_reconstruct_1d_strided", "mci_workspace_size_strided",
           "mci_plan_2d", "mci_upsample_2d", "mci_status_string", "mci_last_error", "mci_plan_variants",
           "mci_plan_set_variant", "mci_plan_autotune", "mci_batch_create", "mci_batch_destroy", "mci_batch_sizes",
           "mci_reconstruct_batch", "mci_offgrid_plan", "mci_offgrid_destroy", "mci_offgrid_info",
           "mci_offgrid_workspace_size", "mci_evaluate_1d", "mci_averaged_error_workspace_size",
           "mci_averaged_error", "mci_error_bound", "mci_plan_omega", "mci_averaged_error_noalloc"]

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
    lib.mci_plan_kernel_name.argtypes = [vp, ctypes.c_char_p, sz]
    lib.mci_plan_kernel_name.restype = i32
    lib.mci_workspace_size.argtypes = [vp, i64, P(sz)]
    lib.mci_reconstruct_1d.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    lib.mci_reconstruct_1d_strided.argtypes = [vp, vp, i64, vp, i64, i64, vp, sz, vp]
    lib.mci_workspace_size_strided.argtypes = [vp, i64, P(sz)]
    lib.mci_plan_2d.argtypes = [P(mci_plan2d_desc), i32, P(vp)]
    lib.mci_upsample_2d.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    lib.mci_status_string.argtypes = [i32]
    lib.mci_status_string.restype = ctypes.c_char_p
    lib.mci_last_error.argtypes = []
    lib.mci_last_error.restype = ctypes.c_char_p
    lib.mci_plan_variants.argtypes = [vp, P(ctypes.c_uint32)]
    lib.mci_plan_set_variant.argtypes = [vp, i32]
    lib.mci_plan_autotune.argtypes = [vp, i64, ctypes.c_char_p, P(mci_tune_result)]
    lib.mci_batch_create.argtypes = [P(mci_batch_item), i64, i32, P(vp)]
    lib.mci_batch_destroy.argtypes = [vp]
    lib.mci_batch_sizes.argtypes = [vp, P(i64), P(i64), P(sz)]
    lib.mci_reconstruct_batch.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.mci_offgrid_plan.argtypes = [P(mci_plan_desc), i32, i32, P(vp)]
    lib.mci_offgrid_destroy.argtypes = [vp]
    lib.mci_offgrid_info.argtypes = [vp, P(i64), P(ctypes.c_int32), P(ctypes.c_double), P(vp)]
    lib.mci_offgrid_workspace_size.argtypes = [vp, i64, i64, P(sz)]
    lib.mci_evaluate_1d.argtypes = [vp, vp, vp, i64, i32, vp, i64, vp, sz, vp]
    lib.mci_averaged_error_workspace_size.argtypes = [i32, i64, i32, P(sz)]
    lib.mci_averaged_error.argtypes = [P(vp), i32, vp, i64, i64, i64, i32, vp, vp, vp, sz, vp]
    lib.mci_error_bound.argtypes = [P(vp), i32, vp, i64, i64, i64, i32, vp, vp, sz, vp]
    lib.mci_plan_omega.argtypes = [vp, P(ctypes.c_double), i32]
    lib.mci_averaged_error_noalloc.argtypes = [P(vp), i32, vp, i64, i64, i64, i32, vp, vp, vp]
    for name in ("mci_offgrid_plan", "mci_offgrid_destroy", "mci_offgrid_info", "mci_offgrid_workspace_size",
                 "mci_evaluate_1d", "mci_averaged_error_workspace_size", "mci_averaged_error", "mci_error_bound",
                 "mci_plan_omega", "mci_averaged_error_noalloc"):
        getattr(lib, name).restype = i32
    for name in ("mci_plan", "mci_plan_destroy", "mci_plan_info", "mci_workspace_size", "mci_reconstruct_1d",
                 "mci_reconstruct_1d_strided", "mci_workspace_size_strided",
                 "mci_plan_2d", "mci_upsample_2d", "mci_plan_variants", "mci_plan_set_variant", "mci_plan_autotune",
                 "mci_batch_create", "mci_batch_destroy", "mci_batch_sizes", "mci_reconstruct_batch"):
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


def mci_plan_kernel_name(plan: int) -> str:
    buf = ctypes.create_string_buffer(256)
    check(load().mci_plan_kernel_name(plan, buf, 256), "mci_plan_kernel_name")
    return buf.value.decode()


def mci_workspace_size(plan: int, batch: int) -> int:
    n = ctypes.c_size_t()
    check(load().mci_workspace_size(plan, batch, ctypes.byref(n)), "mci_workspace_size")
    return n.value


def mci_reconstruct_1d(plan: int, g_ptr: int, y_ptr: int, batch: int, ws_ptr: int, ws_bytes: int,
                       stream: int) -> None:
    check(load().mci_reconstruct_1d(plan, g_ptr, y_ptr, batch, ws_ptr, ws_bytes, stream), "mci_reconstruct_1d")


def mci_workspace_size_strided(plan: int, batch: int) -> int:
    n = ctypes.c_size_t()
    check(load().mci_workspace_size_strided(plan, batch, ctypes.byref(n)), "mci_workspace_size_strided")
    return n.value


def mci_reconstruct_1d_strided(plan: int, g_ptr: int, ld_g: int, y_ptr: int, ld_y: int, batch: int, ws_ptr: int,
                               ws_bytes: int, stream: int) -> None:
    check(load().mci_reconstruct_1d_strided(plan, g_ptr, ld_g, y_ptr, ld_y, batch, ws_ptr, ws_bytes, stream),
          "mci_reconstruct_1d_strided")


def mci_plan_2d(desc: mci_plan2d_desc, device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().mci_plan_2d(ctypes.byref(desc), device, ctypes.byref(h)), "mci_plan_2d")
    return h.value


def mci_upsample_2d(plan: int, lr_ptr: int, hr_ptr: int, batch: int, ws_ptr: int, ws_bytes: int,
                    stream: int) -> None:
    check(load().mci_upsample_2d(plan, lr_ptr, hr_ptr, batch, ws_ptr, ws_bytes, stream), "mci_upsample_2d")


def mci_plan_variants(plan: int) -> int:
    m = ctypes.c_uint32()
    check(load().mci_plan_variants(plan, ctypes.byref(m)), "mci_plan_variants")
    return m.value


def mci_plan_set_variant(plan: int, variant: int) -> None:
    check(load().mci_plan_set_variant(plan, variant), "mci_plan_set_variant")


def mci_plan_autotune(plan: int, batch: int, cache_path: str | None = None) -> mci_tune_result:
    r = mci_tune_result()
    path = cache_path.encode() if cache_path else None
    check(load().mci_plan_autotune(plan, batch, path, ctypes.byref(r)), "mci_plan_autotune")
    return r


def mci_batch_create(items, lanes: int = 0) -> int:
    """items: sequence of (plan handle, in_off, out_off)."""
    arr = (mci_batch_item * max(1, len(items)))()
    for k, (p, i, o) in enumerate(items):
        arr[k].plan, arr[k].in_off, arr[k].out_off = p, i, o
    h = ctypes.c_void_p()
    check(load().mci_batch_create(arr, len(items), lanes, ctypes.byref(h)), "mci_batch_create")
    return h.value


def mci_batch_destroy(batch: int) -> None:
    check(load().mci_batch_destroy(batch), "mci_batch_destroy")


def mci_batch_sizes(batch: int):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    check(load().mci_batch_sizes(batch, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "mci_batch_sizes")
    return a.value, b.value, c.value


def mci_reconstruct_batch(batch: int, in_ptr: int, out_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(load().mci_reconstruct_batch(batch, in_ptr, out_ptr, ws_ptr, ws_bytes, stream), "mci_reconstruct_batch")


def mci_offgrid_plan(desc: mci_plan_desc, width: int = 0, device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().mci_offgrid_plan(ctypes.byref(desc), width, device, ctypes.byref(h)), "mci_offgrid_plan")
    return h.value


def mci_offgrid_destroy(plan: int) -> None:
    check(load().mci_offgrid_destroy(plan), "mci_offgrid_destroy")


def mci_offgrid_info(plan: int):
    """(grid length L, width w, beta, handle of the grid plan)"""
    L, w, beta, g = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_void_p()
    check(load().mci_offgrid_info(plan, ctypes.byref(L), ctypes.byref(w), ctypes.byref(beta), ctypes.byref(g)),
          "mci_offgrid_info")
    return L.value, w.value, beta.value, g.value


def mci_offgrid_workspace_size(plan: int, batch: int, n_t: int) -> int:
    n = ctypes.c_size_t()
    check(load().mci_offgrid_workspace_size(plan, batch, n_t, ctypes.byref(n)), "mci_offgrid_workspace_size")
    return n.value


def mci_evaluate_1d(plan: int, g_ptr: int, t_ptr: int, n_t: int, t_shared: bool, y_ptr: int, batch: int,
                    ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(load().mci_evaluate_1d(plan, g_ptr, t_ptr, n_t, 1 if t_shared else 0, y_ptr, batch, ws_ptr, ws_bytes,
                                 stream), "mci_evaluate_1d")


def mci_averaged_error_workspace_size(n_plans: int, n_span: int, precision: int) -> int:
    n = ctypes.c_size_t()
    check(load().mci_averaged_error_workspace_size(n_plans, n_span, precision, ctypes.byref(n)),
          "mci_averaged_error_workspace_size")
    return n.value


def mci_averaged_error(plans, a_ptr: int, n_lo: int, n_span: int, n_sig: int, precision: int, eps_ptr: int,
                       best_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    arr = (ctypes.c_void_p * max(1, len(plans)))(*plans)
    check(load().mci_averaged_error(arr, len(plans), a_ptr, n_lo, n_span, n_sig, precision, eps_ptr, best_ptr,
                                    ws_ptr, ws_bytes, stream), "mci_averaged_error")


def mci_error_bound(plans, a_ptr: int, n_lo: int, n_span: int, n_sig: int, precision: int, bound_ptr: int,
                    ws_ptr: int, ws_bytes: int, stream: int) -> None:
    arr = (ctypes.c_void_p * max(1, len(plans)))(*plans)
    check(load().mci_error_bound(arr, len(plans), a_ptr, n_lo, n_span, n_sig, precision, bound_ptr, ws_ptr,
                                 ws_bytes, stream), "mci_error_bound")


def mci_averaged_error_noalloc(plans, a_ptr: int, n_lo: int, n_span: int, n_sig: int, precision: int, eps_ptr: int,
                               best_ptr: int, stream: int) -> None:
    arr = (ctypes.c_void_p * max(1, len(plans)))(*plans)
    check(load().mci_averaged_error_noalloc(arr, len(plans), a_ptr, n_lo, n_span, n_sig, precision, eps_ptr,
                                            best_ptr, stream), "mci_averaged_error_noalloc")


def mci_plan_omega(plan, M: int):
    out = (ctypes.c_double * max(1, M))()
    check(load().mci_plan_omega(plan, out, M), "mci_plan_omega")
    return list(out)[:M]


# ----------------------------------------------------------------------------- refiner
REFINER_EXPORTS = ["mci_refiner_create", "mci_refiner_destroy", "mci_refiner_num_params", "mci_refiner_get_params",
                   "mci_refiner_set_params", "mci_refiner_get_grads", "mci_refiner_workspace_size",
                   "mci_refiner_forward", "mci_refiner_backward", "mci_refiner_train_step", "mci_refiner_last_error",
                   "mci_refiner_state_size", "mci_refiner_save_state", "mci_refiner_load_state"]
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
    lib.mci_refiner_state_size.argtypes = []
    lib.mci_refiner_state_size.restype = sz
    lib.mci_refiner_save_state.argtypes = [vp, vp, sz]
    lib.mci_refiner_load_state.argtypes = [vp, vp, sz]
    for n in ("mci_refiner_create", "mci_refiner_destroy", "mci_refiner_get_params", "mci_refiner_set_params",
              "mci_refiner_get_grads", "mci_refiner_workspace_size", "mci_refiner_forward", "mci_refiner_backward",
              "mci_refiner_train_step", "mci_refiner_save_state", "mci_refiner_load_state"):
        getattr(lib, n).restype = i32
    lib._refiner_ready = True
    return lib


def rcheck(status: int, where: str):
    if status != 0:
        raise MCIError(status, where, load_refiner().mci_refiner_last_error().decode(errors="replace"))
