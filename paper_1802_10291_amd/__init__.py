"""FFT multichannel interpolation (Cheng & Kou, arXiv:1802.10291) on MI355X.

Python face of libmci (include/mci.h).  Every step of the reconstruction runs in the
library's HIP kernels; this module only builds descriptors, allocates the caller-side
workspace with PyTorch and passes device pointers and the current HIP stream.

    plan = Plan1D(N=1366, n_out=16384, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)])
    y = plan.reconstruct(g)          # g: float32 cuda tensor [batch, 3, 1366]

    up = Plan2D(h=256, w=256, scale=2)
    hr = up.upsample(lr)             # lr: float32 cuda tensor [batch, 256, 256]
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple, Union

import numpy as np

from . import _lib
from ._lib import (  # noqa: F401  (the C-ABI names, re-exported)
    MCIError, mci_plan, mci_plan_destroy, mci_plan_info, mci_workspace_size, mci_reconstruct_1d, mci_plan_2d,
    mci_reconstruct_1d_strided, mci_workspace_size_strided,
    mci_upsample_2d, mci_plan_variants, mci_plan_set_variant, mci_plan_autotune, mci_batch_create,
    mci_batch_destroy, mci_batch_sizes, mci_reconstruct_batch, VARIANT_NAMES,
)

def _batch_stride(t):
    """Elements between consecutive items of t's first dimension when every item is
    contiguous (None otherwise)."""
    if t.dim() == 0:
        return None
    inner = 1
    for d in t.shape[1:]:
        inner *= d
    if t.is_contiguous():
        return inner
    if t.shape[0] == 0 or not t[0].is_contiguous():
        return None
    return t.stride(0) if t.shape[0] > 1 else inner


_KINDS = {"deriv": _lib.MCI_MULT_DERIV, "hilbert": _lib.MCI_MULT_HILBERT, "table": _lib.MCI_MULT_TABLE}
_OPS = {"identity": _lib.MCI_OUT_IDENTITY, "hilbert": _lib.MCI_OUT_HILBERT, "deriv": _lib.MCI_OUT_DERIV}

Channel = Union[Tuple[str, int], Tuple[str, np.ndarray]]


def _torch():
    import torch
    return torch


def _stream_handle(device) -> int:
    torch = _torch()
    return int(torch.cuda.current_stream(device).cuda_stream)


class _Workspaces:
    """Caller-side workspaces of one library object, one buffer per stream.  Calls queued on
    different streams never share scratch memory, and each buffer is allocated (or replaced
    when it must grow) while its own stream is current, so PyTorch's caching allocator hands
    it out again only in that stream's order, after the kernels queued on it."""

    def __init__(self, device: int):
        self.device = device
        self.bufs = {}

    def get(self, need: int):
        torch = _torch()
        key = _stream_handle(self.device)
        buf = self.bufs.get(key)
        if buf is None or buf.numel() < need:
            buf = torch.empty(max(int(need), 1), dtype=torch.uint8, device=f"cuda:{self.device}")
            self.bufs[key] = buf
        return buf


class _Variants:
    """Kernel variants and the autotuner (``mci_plan_variants`` / ``mci_plan_set_variant`` /
    ``mci_plan_autotune``), shared by 1-D and 2-D plans."""

    def variants(self):
        m = mci_plan_variants(self.handle)
        return [VARIANT_NAMES[v] for v in range(len(VARIANT_NAMES)) if m >> v & 1]

    @property
    def variant(self) -> str:
        return VARIANT_NAMES[mci_plan_info(self.handle).variant]

    def set_variant(self, name: str) -> None:
        mci_plan_set_variant(self.handle, VARIANT_NAMES.index(name))

    def autotune(self, batch: int, cache_path: Optional[str] = None):
        """Time every variant at this batch, keep the fastest; returns (name, {name: ms}, from_cache)."""
        r = mci_plan_autotune(self.handle, batch, cache_path)
        ms = {VARIANT_NAMES[v]: r.ms[v] for v in range(len(VARIANT_NAMES)) if r.ms[v] >= 0}
        return VARIANT_NAMES[r.variant], ms, bool(r.from_cache)

    def instance_sizes(self) -> Tuple[int, int]:
        """Elements of one instance's input and output."""
        raise NotImplementedError

    def kernel_name(self) -> str:
        """The kernels of the active variant (``mci_plan_kernel_name``)."""
        return _lib.mci_plan_kernel_name(self.handle)


def _desc_1d(N, n_out, channels, ops, n1, real, precision, storage, allow_singular_zero, cond_max):
    """An mci_plan_desc, and the host channel tables it points to (kept alive by the caller)."""
    d = _lib.mci_plan_desc()
    d.M = len(channels)
    d.n_ops = len(ops)
    d.N = int(N)
    d.n1 = _lib.MCI_N1_DEFAULT if n1 is None else int(n1)
    d.n_out = int(n_out)
    tables = []
    for k, (kind, arg) in enumerate(channels):
        d.ch[k].kind = _KINDS[kind]
        if kind == "table":
            t = np.ascontiguousarray(np.asarray(arg, dtype=np.complex128).ravel().view(np.float64))
            tables.append(t)
            d.ch[k].table = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            d.ch[k].order = int(arg)
    for o, (op, order) in enumerate(ops):
        d.ops[o] = _OPS[op]
        d.op_orders[o] = int(order)
    d.real_io = 1 if real else 0
    d.precision = {"f32": _lib.MCI_F32, "f64": _lib.MCI_F64}[precision]
    d.storage = {"native": _lib.MCI_STORE_NATIVE, "f16": _lib.MCI_STORE_F16}[storage]
    d.flags = _lib.MCI_ALLOW_SINGULAR_ZERO if allow_singular_zero else 0
    d.cond_max = float(cond_max)
    return d, tables


class Plan1D(_Variants):
    """A 1-D reconstruction plan (``mci_plan``).

    channels: list of ("deriv", order) | ("hilbert", 0) | ("table", complex array of
    length M*N with b(n) for n in [n1, n1 + M N)).  ops: list of ("identity", 0) |
    ("hilbert", 0) | ("deriv", order).
    """

    def __init__(self, N: int, n_out: int, channels: Sequence[Channel], ops: Sequence[Tuple[str, int]] = (("identity", 0),),
                 n1: Optional[int] = None, real: bool = True, precision: str = "f32", storage: str = "native",
                 allow_singular_zero: bool = False, cond_max: float = 0.0, device: int = 0):
        d, self._tables = _desc_1d(N, n_out, channels, ops, n1, real, precision, storage, allow_singular_zero,
                                   cond_max)
        self.desc = d
        self.M, self.N, self.n_out, self.n_ops, self.real = d.M, int(N), int(n_out), d.n_ops, real
        self.precision, self.storage, self.device = precision, storage, device
        self.handle = mci_plan(d, device)
        self._ws = _Workspaces(device)

    @property
    def info(self):
        return mci_plan_info(self.handle)

    def omega(self):
        """Omega_1..Omega_M of the error bound (``mci_plan_omega``, after Theorem 4.4)."""
        return _lib.mci_plan_omega(self.handle, self.M)

    def instance_sizes(self) -> Tuple[int, int]:
        c = 1 if self.real else 2
        return self.M * self.N * c, self.n_ops * self.n_out * c

    def io_dtype(self):
        torch = _torch()
        if self.storage == "f16":
            return torch.float16
        return torch.float64 if self.precision == "f64" else torch.float32

    def workspace(self, batch: int):
        """(buffer, bytes) of the workspace for the current stream (None when none is needed)."""
        need = mci_workspace_size(self.handle, batch)
        return (self._ws.get(need) if need else None), need

    def reconstruct(self, g, out=None):
        """g: cuda tensor [batch, M, N] (real) or [batch, M, N, 2] (complex, re/im).
        Returns [batch, n_ops, n_out] (or [..., 2]), or fills `out`.  Each signal of g and out
        must be contiguous; the batch dimension may be strided (signals spaced a multiple of 4
        elements apart, e.g. a slice of longer rows), which runs mci_reconstruct_1d_strided."""
        torch = _torch()
        if not g.is_cuda:
            raise ValueError("g must be a device tensor")
        tail = (self.M, self.N) if self.real else (self.M, self.N, 2)
        if tuple(g.shape[1:]) != tail or g.dtype != self.io_dtype() or _batch_stride(g) is None:
            raise ValueError(f"g must be {self.io_dtype()} [batch, {', '.join(map(str, tail))}] "
                             "with contiguous signals")
        batch = g.shape[0]
        shape = (batch, self.n_ops, self.n_out) if self.real else (batch, self.n_ops, self.n_out, 2)
        if out is None:
            out = torch.empty(shape, dtype=self.io_dtype(), device=g.device)
        elif tuple(out.shape) != shape or out.dtype != self.io_dtype() or _batch_stride(out) is None:
            raise ValueError("bad out tensor")
        if g.is_contiguous() and out.is_contiguous():
            ws, need = self.workspace(batch)
            mci_reconstruct_1d(self.handle, g.data_ptr(), out.data_ptr(), batch,
                               ws.data_ptr() if ws is not None else 0, need, _stream_handle(g.device))
            return out
        need = mci_workspace_size_strided(self.handle, batch)
        ws = self._ws.get(need) if need else None
        mci_reconstruct_1d_strided(self.handle, g.data_ptr(), _batch_stride(g), out.data_ptr(), _batch_stride(out),
                                   batch, ws.data_ptr() if ws is not None else 0, need, _stream_handle(g.device))
        return out

    def close(self):
        if getattr(self, "handle", None):
            mci_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class OffGrid:
    """Evaluation of the reconstruction at arbitrary points t (``mci_offgrid_plan`` /
    ``mci_evaluate_1d``): the same channels, band and output operators as :class:`Plan1D`,
    evaluated by a nonuniform FFT of kernel width ``width`` (0: chosen for an error near
    4e-7 in FP32 plans, 1e-12 in FP64 plans)."""

    def __init__(self, N: int, channels: Sequence[Channel], ops: Sequence[Tuple[str, int]] = (("identity", 0),),
                 n1: Optional[int] = None, real: bool = True, precision: str = "f32", width: int = 0,
                 allow_singular_zero: bool = False, cond_max: float = 0.0, device: int = 0):
        d, self._tables = _desc_1d(N, 1, channels, ops, n1, real, precision, "native", allow_singular_zero,
                                   cond_max)
        self.M, self.N, self.n_ops, self.real = d.M, int(N), d.n_ops, real
        self.precision, self.device = precision, device
        self.handle = _lib.mci_offgrid_plan(d, width, device)
        self.grid_len, self.width, self.beta, grid_plan = _lib.mci_offgrid_info(self.handle)
        self._ws = _Workspaces(device)

    def io_dtype(self):
        torch = _torch()
        return torch.float64 if self.precision == "f64" else torch.float32

    def evaluate(self, g, t, out=None):
        """g: cuda tensor [batch, M, N] (real) or [batch, M, N, 2]; t: float64 cuda tensor
        [n_t] (the same points for every signal) or [batch, n_t].  Returns
        [batch, n_ops, n_t] (or [..., 2])."""
        torch = _torch()
        if not g.is_cuda or not t.is_cuda:
            raise ValueError("g and t must be device tensors")
        tail = (self.M, self.N) if self.real else (self.M, self.N, 2)
        if tuple(g.shape[1:]) != tail or g.dtype != self.io_dtype() or not g.is_contiguous():
            raise ValueError(f"g must be contiguous {self.io_dtype()} [batch, {', '.join(map(str, tail))}]")
        batch = g.shape[0]
        if t.dtype != torch.float64 or not t.is_contiguous() or t.dim() not in (1, 2) or \
                (t.dim() == 2 and t.shape[0] != batch):
            raise ValueError("t must be contiguous float64 [n_t] or [batch, n_t]")
        n_t = t.shape[-1]
        shape = (batch, self.n_ops, n_t) if self.real else (batch, self.n_ops, n_t, 2)
        if out is None:
            out = torch.empty(shape, dtype=self.io_dtype(), device=g.device)
        elif tuple(out.shape) != shape or out.dtype != self.io_dtype() or not out.is_contiguous():
            raise ValueError("bad out tensor")
        need = _lib.mci_offgrid_workspace_size(self.handle, batch, n_t)
        ws = self._ws.get(need)
        _lib.mci_evaluate_1d(self.handle, g.data_ptr(), t.data_ptr(), n_t, t.dim() == 1, out.data_ptr(), batch,
                             ws.data_ptr(), need, _stream_handle(g.device))
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.mci_offgrid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def averaged_error(plans: Sequence["Plan1D"], a, n_lo: int):
    """Averaged approximation error (Theorem 4.4) of every signal under every plan
    (``mci_averaged_error``).  a: complex64 / complex128 cuda tensor [n_sig, n_span] with
    a[s, i] = a_s(n_lo + i).  Returns (eps float64 [n_sig, n_plans], best int32 [n_sig])."""
    torch = _torch()
    if not a.is_cuda or a.dim() != 2 or not a.is_contiguous() or a.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("a must be a contiguous complex64/complex128 cuda tensor [n_sig, n_span]")
    prec = _lib.MCI_F64 if a.dtype == torch.complex128 else _lib.MCI_F32
    n_sig, n_span = a.shape
    eps = torch.empty((n_sig, len(plans)), dtype=torch.float64, device=a.device)
    best = torch.empty((n_sig,), dtype=torch.int32, device=a.device)
    need = _lib.mci_averaged_error_workspace_size(len(plans), n_span, prec)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=a.device)
    _lib.mci_averaged_error([p.handle for p in plans], a.data_ptr(), int(n_lo), n_span, n_sig, prec, eps.data_ptr(),
                            best.data_ptr(), ws.data_ptr(), need, _stream_handle(a.device))
    return eps, best


def error_bound(plans: Sequence["Plan1D"], a, n_lo: int):
    """The bound of eq. errorestimate on the averaged error of every signal under every plan
    (``mci_error_bound``); a as for :func:`averaged_error`.  Returns float64 [n_sig, n_plans]."""
    torch = _torch()
    if not a.is_cuda or a.dim() != 2 or not a.is_contiguous() or a.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("a must be a contiguous complex64/complex128 cuda tensor [n_sig, n_span]")
    prec = _lib.MCI_F64 if a.dtype == torch.complex128 else _lib.MCI_F32
    n_sig, n_span = a.shape
    bound = torch.empty((n_sig, len(plans)), dtype=torch.float64, device=a.device)
    need = _lib.mci_averaged_error_workspace_size(len(plans), n_span, prec)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=a.device)
    _lib.mci_error_bound([p.handle for p in plans], a.data_ptr(), int(n_lo), n_span, n_sig, prec, bound.data_ptr(),
                         ws.data_ptr(), need, _stream_handle(a.device))
    return bound


class Plan2D(_Variants):
    """A 2-D separable upsampling plan (``mci_plan_2d``): lr [batch, h, w] -> hr [batch, s h, s w],
    with channels {x, Dx} (channels=2) or {x, Dx, D2x} (channels=3) per line."""

    def __init__(self, h: int, w: int, scale: int, precision: str = "f32", storage: str = "native", device: int = 0,
                 channels: int = 2):
        d = _lib.mci_plan2d_desc()
        d.h, d.w, d.scale = int(h), int(w), int(scale)
        d.channels = int(channels)
        d.precision = {"f32": _lib.MCI_F32, "f64": _lib.MCI_F64}[precision]
        d.storage = {"native": _lib.MCI_STORE_NATIVE, "f16": _lib.MCI_STORE_F16}[storage]
        self.desc = d
        self.h, self.w, self.scale = int(h), int(w), int(scale)
        self.precision, self.storage, self.device = precision, storage, device
        self.handle = mci_plan_2d(d, device)
        self._ws = _Workspaces(device)

    @property
    def info(self):
        return mci_plan_info(self.handle)

    def instance_sizes(self) -> Tuple[int, int]:
        return self.h * self.w, self.scale * self.scale * self.h * self.w

    def io_dtype(self):
        torch = _torch()
        if self.storage == "f16":
            return torch.float16
        return torch.float64 if self.precision == "f64" else torch.float32

    def workspace(self, batch: int):
        """(buffer, bytes) of the workspace for the current stream (None when none is needed)."""
        need = mci_workspace_size(self.handle, batch)
        return (self._ws.get(need) if need else None), need

    def upsample(self, lr, out=None):
        torch = _torch()
        if not lr.is_cuda or tuple(lr.shape[1:]) != (self.h, self.w) or lr.dtype != self.io_dtype() \
                or not lr.is_contiguous():
            raise ValueError(f"lr must be a contiguous device {self.io_dtype()} tensor [batch, {self.h}, {self.w}]")
        batch = lr.shape[0]
        shape = (batch, self.scale * self.h, self.scale * self.w)
        if out is None:
            out = torch.empty(shape, dtype=self.io_dtype(), device=lr.device)
        elif tuple(out.shape) != shape or out.dtype != self.io_dtype() or not out.is_contiguous():
            raise ValueError("bad out tensor")
        ws, need = self.workspace(batch)
        mci_upsample_2d(self.handle, lr.data_ptr(), out.data_ptr(), batch, ws.data_ptr() if ws is not None else 0,
                        need, _stream_handle(lr.device))
        return out

    def close(self):
        if getattr(self, "handle", None):
            mci_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Uneven batch (``mci_batch_*``): instances of several plans (1-D lengths, channel counts,
    2-D sizes) over ragged packed buffers, reconstructed by one call.

    instances: sequence of plans, one per instance (a plan may repeat).  Instance k's input
    and output sit at ``in_offsets[k]`` / ``out_offsets[k]`` of the flat packed buffers, each
    rounded up to ``align`` elements, in the order given (or pass explicit offsets).
    """

    def __init__(self, instances: Sequence, lanes: int = 16, align: int = 64, offsets=None):
        self.plans = list(instances)
        if offsets is None:
            ins, outs, i, o = [], [], 0, 0
            for p in self.plans:
                ni, no = p.instance_sizes()
                ins.append(i)
                outs.append(o)
                i += -(-ni // align) * align
                o += -(-no // align) * align
            offsets = (ins, outs)
        self.in_offsets, self.out_offsets = list(offsets[0]), list(offsets[1])
        self.handle = mci_batch_create([(p.handle, i, o) for p, i, o in
                                        zip(self.plans, self.in_offsets, self.out_offsets)], lanes)
        self.in_elems, self.out_elems, self.ws_bytes = mci_batch_sizes(self.handle)
        self.device = self.plans[0].device if self.plans else 0
        self._ws = _Workspaces(self.device)

    def dtype(self):
        return self.plans[0].io_dtype()

    def workspace(self):
        """(buffer, bytes) of the workspace for the current stream (None when none is needed)."""
        _, _, need = mci_batch_sizes(self.handle)
        return (self._ws.get(need) if need else None), need

    def run(self, packed_in, packed_out=None):
        """packed_in: flat device tensor of >= in_elems elements; returns the packed output."""
        torch = _torch()
        if not packed_in.is_cuda or packed_in.dtype != self.dtype() or packed_in.numel() < self.in_elems \
                or not packed_in.is_contiguous():
            raise ValueError(f"packed input must be a contiguous device {self.dtype()} tensor of >= {self.in_elems}")
        if packed_out is None:
            packed_out = torch.empty(self.out_elems, dtype=self.dtype(), device=packed_in.device)
        elif packed_out.numel() < self.out_elems or packed_out.dtype != self.dtype() or not packed_out.is_contiguous():
            raise ValueError("bad packed output")
        ws, need = self.workspace()
        mci_reconstruct_batch(self.handle, packed_in.data_ptr(), packed_out.data_ptr(),
                              ws.data_ptr() if ws is not None else 0, need, _stream_handle(packed_in.device))
        return packed_out

    def close(self):
        if getattr(self, "handle", None):
            mci_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Refiner:
    """Learned residual refiner y = u + CNN(u) (``mci_refiner_*``): BF16 MFMA kernels, FP32
    master weights, Adam.  Images are float32 cuda tensors [B, 3, H, W]."""

    def __init__(self, seed: int = 0, device: int = 0):
        lib = _lib.load_refiner()
        h = ctypes.c_void_p()
        _lib.rcheck(lib.mci_refiner_create(device, seed, ctypes.byref(h)), "mci_refiner_create")
        self.handle, self.device = h.value, device
        self.n_params = int(lib.mci_refiner_num_params())
        self._ws = _Workspaces(device)
        self._lp = None

    def _workspace(self, B, H, W):
        n = ctypes.c_size_t()
        _lib.rcheck(_lib.load_refiner().mci_refiner_workspace_size(B, H, W, ctypes.byref(n)), "workspace_size")
        return self._ws.get(n.value), n.value

    @staticmethod
    def _check_img(t):
        if not t.is_cuda or t.dtype != _torch().float32 or t.dim() != 4 or t.shape[1] != 3 or not t.is_contiguous():
            raise ValueError("images must be contiguous float32 cuda tensors [B, 3, H, W]")

    def get_params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        tau = ctypes.c_float()
        _lib.rcheck(_lib.load_refiner().mci_refiner_get_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                               ctypes.byref(tau)), "get_params")
        return p, tau.value

    def set_params(self, params, tau: float = 0.0):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError("wrong parameter count")
        _lib.rcheck(_lib.load_refiner().mci_refiner_set_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                               float(tau)), "set_params")

    def save_state(self) -> bytes:
        """Checkpoint of the training state (``mci_refiner_save_state``): parameters, Adam
        moments and step count, fallback bound."""
        lib = _lib.load_refiner()
        n = int(lib.mci_refiner_state_size())
        buf = ctypes.create_string_buffer(n)
        _lib.rcheck(lib.mci_refiner_save_state(self.handle, buf, n), "mci_refiner_save_state")
        return buf.raw

    def load_state(self, state: bytes) -> None:
        """Restore a checkpoint written by :meth:`save_state` (``mci_refiner_load_state``)."""
        lib = _lib.load_refiner()
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _lib.rcheck(lib.mci_refiner_load_state(self.handle, buf, len(state)), "mci_refiner_load_state")

    def get_grads(self):
        g = np.empty(self.n_params, dtype=np.float32)
        _lib.rcheck(_lib.load_refiner().mci_refiner_get_grads(self.handle, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "get_grads")
        return g

    def forward(self, u, fallback: bool = False, out=None):
        """Returns (y, ratio, used): ratio[b] = ||y_b - u_b|| / ||u_b||; with fallback, images
        above the stored bound get y_b = u_b and used[b] = 0."""
        torch = _torch()
        self._check_img(u)
        B, _, H, W = u.shape
        y = torch.empty_like(u) if out is None else out
        ratio = torch.empty(B, dtype=torch.float32, device=u.device)
        used = torch.ones(B, dtype=torch.int32, device=u.device)
        ws, n = self._workspace(B, H, W)
        _lib.rcheck(_lib.load_refiner().mci_refiner_forward(self.handle, u.data_ptr(), y.data_ptr(), B, H, W, int(fallback),
                                                            ratio.data_ptr(), used.data_ptr(), ws.data_ptr(), n,
                                                            _stream_handle(u.device)), "mci_refiner_forward")
        return y, ratio, used

    def _loss_call(self, fn, u, hr, *extra):
        torch = _torch()
        self._check_img(u)
        self._check_img(hr)
        B, _, H, W = u.shape
        if self._lp is None:
            self._lp = torch.zeros(4096, dtype=torch.float32, device=u.device)
        ws, n = self._workspace(B, H, W)
        nparts = ctypes.c_int()
        _lib.rcheck(fn(self.handle, u.data_ptr(), hr.data_ptr(), B, H, W, *extra, self._lp.data_ptr(),
                       ctypes.byref(nparts), ws.data_ptr(), n, _stream_handle(u.device)), fn.__name__)
        return self._lp[: nparts.value], B * 3 * H * W

    def backward(self, u, hr):
        """Fills the gradient of mean((u + CNN(u) - hr)^2); returns the loss (device scalar)."""
        parts, count = self._loss_call(_lib.load_refiner().mci_refiner_backward, u, hr)
        return parts.sum() / count

    def train_step(self, u, hr, lr: float = 1e-3):
        parts, count = self._loss_call(_lib.load_refiner().mci_refiner_train_step, u, hr, ctypes.c_float(lr))
        return parts.sum() / count

    def close(self):
        if getattr(self, "handle", None):
            _lib.load_refiner().mci_refiner_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upsample_rgb(plan: "Plan2D", lr_rgb, out=None):
    """MCI upsample of RGB images [B, 3, h, w] plane by plane with a Plan2D."""
    B = lr_rgb.shape[0]
    planes = lr_rgb.reshape(B * 3, lr_rgb.shape[2], lr_rgb.shape[3])
    hr = plan.upsample(planes, None if out is None else out.reshape(B * 3, out.shape[2], out.shape[3]))
    return hr.reshape(B, 3, hr.shape[1], hr.shape[2])
