"""Host-side checks of libmci that need no GPU: the library loads, exports every symbol
include/mci.h declares, its ctypes structures match the header's layout, and
descriptor validation rejects bad input before any device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mci.h")


def _lib():
    from paper_1802_10291_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libmci.so not built")
    return L


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(mci_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for n in ("mci_plan", "mci_reconstruct_1d", "mci_upsample_2d", "mci_plan_2d", "mci_plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared_functions()) <= set(L.EXPORTS)


def test_struct_sizes_match_c_layout():
    L = _lib()
    # int32 M, n_ops; int64 N, n1, n_out; 4 x {int32, int32, ptr}; 4 + 4 int32; 4 int32 fields; double
    assert ctypes.sizeof(L.mci_channel) == 16
    assert ctypes.sizeof(L.mci_plan_desc) == 8 + 24 + 64 + 32 + 16 + 8
    assert L.mci_plan_desc.cond_max.offset == 144
    assert ctypes.sizeof(L.mci_plan_info_t) == 56
    assert ctypes.sizeof(L.mci_plan2d_desc) == 24


def test_status_strings():
    L = _lib()
    lib = L.load()
    for code, name in L.STATUS.items():
        assert lib.mci_status_string(code).decode() == name


def _desc(L, **kw):
    d = L.mci_plan_desc()
    d.M, d.n_ops, d.N, d.n1, d.n_out = 2, 1, 16, L.MCI_N1_DEFAULT, 64
    d.ch[0].kind, d.ch[0].order = L.MCI_MULT_DERIV, 0
    d.ch[1].kind, d.ch[1].order = L.MCI_MULT_DERIV, 1
    d.ops[0] = L.MCI_OUT_IDENTITY
    d.real_io, d.precision, d.storage = 1, L.MCI_F32, L.MCI_STORE_NATIVE
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value", [("M", 0), ("M", 5), ("n_ops", 0), ("N", 0), ("n_out", 0),
                                         ("precision", 7), ("storage", 9), ("real_io", 2), ("flags", 8)])
def test_invalid_descriptors_rejected_without_device(field, value):
    L = _lib()
    lib = L.load()
    d = _desc(L, **{field: value})
    h = ctypes.c_void_p()
    assert lib.mci_plan(ctypes.byref(d), 0, ctypes.byref(h)) == 1   # MCI_E_INVALID_ARG
    assert h.value is None
    assert lib.mci_last_error().decode()


def test_invalid_channel_kinds_rejected():
    L = _lib()
    lib = L.load()
    h = ctypes.c_void_p()
    d = _desc(L)
    d.ch[1].kind = 9
    assert lib.mci_plan(ctypes.byref(d), 0, ctypes.byref(h)) == 1
    d = _desc(L)
    d.ch[1].kind = L.MCI_MULT_TABLE      # table channel without a table
    assert lib.mci_plan(ctypes.byref(d), 0, ctypes.byref(h)) == 1
    d = _desc(L, storage=L.MCI_STORE_F16, precision=L.MCI_F64)
    assert lib.mci_plan(ctypes.byref(d), 0, ctypes.byref(h)) == 1


def test_null_arguments_rejected():
    L = _lib()
    lib = L.load()
    assert lib.mci_plan(None, 0, None) == 1
    assert lib.mci_plan_destroy(None) == 0
    assert lib.mci_reconstruct_1d(None, None, None, 1, None, 0, None) == 1
    assert lib.mci_reconstruct_1d_strided(None, None, 0, None, 0, 1, None, 0, None) == 1
    n = ctypes.c_size_t()
    assert lib.mci_workspace_size(None, 1, ctypes.byref(n)) == 1
    assert lib.mci_workspace_size_strided(None, 1, ctypes.byref(n)) == 1


def test_batch_and_tuner_structs_match_c_layout():
    L = _lib()
    # mci_batch_item: pointer + 2 int64; mci_tune_result: 2 int32 + int64 + 5 doubles
    assert ctypes.sizeof(L.mci_batch_item) == 24
    assert ctypes.sizeof(L.mci_tune_result) == 16 + 8 * L.MCI_NUM_VARIANTS
    assert L.mci_tune_result.ms.offset == 16
    assert L.mci_plan_info_t.variant.offset == 52


def test_batch_and_variant_arguments_rejected_without_device():
    L = _lib()
    lib = L.load()
    h = ctypes.c_void_p()
    items = (L.mci_batch_item * 1)()
    items[0].plan, items[0].in_off, items[0].out_off = None, 0, 0
    assert lib.mci_batch_create(items, 1, 0, ctypes.byref(h)) == 1       # NULL plan
    assert lib.mci_batch_create(items, -1, 0, ctypes.byref(h)) == 1      # negative count
    assert lib.mci_batch_create(items, 0, 17, ctypes.byref(h)) == 1      # lanes out of range
    assert lib.mci_batch_create(items, 0, 0, None) == 1
    assert lib.mci_plan_set_variant(None, 0) == 1
    assert lib.mci_plan_autotune(None, 1, None, None) == 1
    assert lib.mci_reconstruct_batch(None, None, None, None, 0, None) == 1
    # an empty batch needs no device: it is created, sized and run as a no-op
    assert lib.mci_batch_create(items, 0, 0, ctypes.byref(h)) == 0
    a, b, c = ctypes.c_int64(7), ctypes.c_int64(7), ctypes.c_size_t(7)
    assert lib.mci_batch_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == 0
    assert (a.value, b.value, c.value) == (0, 0, 0)
    assert lib.mci_reconstruct_batch(h, None, None, None, 0, None) == 0
    assert lib.mci_batch_destroy(h) == 0


def test_2d_descriptor_channels_validated_without_device():
    L = _lib()
    lib = L.load()
    d = L.mci_plan2d_desc()
    d.h, d.w, d.scale, d.precision, d.storage = 16, 16, 3, L.MCI_F32, L.MCI_STORE_NATIVE
    h = ctypes.c_void_p()
    for bad in (1, 4, -1):
        d.channels = bad
        assert lib.mci_plan_2d(ctypes.byref(d), 0, ctypes.byref(h)) == 1
        assert "channels" in lib.mci_last_error().decode()


def test_offgrid_arguments_rejected_without_device():
    L = _lib()
    lib = L.load()
    h = ctypes.c_void_p()
    d = _desc(L)
    assert lib.mci_offgrid_plan(ctypes.byref(d), 1, 0, ctypes.byref(h)) == 1     # width below 2
    assert lib.mci_offgrid_plan(ctypes.byref(d), 17, 0, ctypes.byref(h)) == 1    # width above 16
    assert h.value is None
    d = _desc(L, storage=L.MCI_STORE_F16)
    assert lib.mci_offgrid_plan(ctypes.byref(d), 0, 0, ctypes.byref(h)) == 4     # MCI_E_UNSUPPORTED
    d = _desc(L, M=0)
    assert lib.mci_offgrid_plan(ctypes.byref(d), 0, 0, ctypes.byref(h)) == 1
    assert lib.mci_offgrid_plan(None, 0, 0, ctypes.byref(h)) == 1
    assert lib.mci_offgrid_plan(ctypes.byref(_desc(L)), 0, 0, None) == 1
    assert lib.mci_offgrid_destroy(None) == 0
    n = ctypes.c_size_t()
    assert lib.mci_offgrid_workspace_size(None, 1, 1, ctypes.byref(n)) == 1
    assert lib.mci_offgrid_info(None, None, None, None, None) == 1
    assert lib.mci_evaluate_1d(None, None, None, 1, 1, None, 1, None, 0, None) == 1


def test_averaged_error_arguments_rejected_without_device():
    L = _lib()
    lib = L.load()
    n = ctypes.c_size_t()
    assert lib.mci_averaged_error_workspace_size(0, 10, 0, ctypes.byref(n)) == 1     # no plans
    assert lib.mci_averaged_error_workspace_size(17, 10, 0, ctypes.byref(n)) == 1    # above 16
    assert lib.mci_averaged_error_workspace_size(3, 10, 5, ctypes.byref(n)) == 1     # precision
    assert lib.mci_averaged_error_workspace_size(3, 10, 1, ctypes.byref(n)) == 0
    assert n.value == 4 * 10 * 8 + (256 - (4 * 10 * 8) % 256) + 256                  # 4 padded rows, FP64, constants
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.mci_averaged_error(arr, 1, None, 0, 10, 1, 0, None, None, None, 0, None) == 1   # NULL plan
    assert lib.mci_averaged_error(None, 1, None, 0, 10, 1, 0, None, None, None, 0, None) == 1
    assert lib.mci_averaged_error(arr, 0, None, 0, 10, 1, 0, None, None, None, 0, None) == 1
    assert lib.mci_error_bound(arr, 1, None, 0, 10, 1, 0, None, None, 0, None) == 1      # NULL plan
    assert lib.mci_error_bound(None, 1, None, 0, 10, 1, 0, None, None, 0, None) == 1
    om = (ctypes.c_double * 4)()
    assert lib.mci_plan_omega(None, om, 4) == 1
