"""FP64 CPU oracle for FFT multichannel interpolation (Cheng & Kou, arXiv:1802.10291).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark import this module.  The product package never imports it and
shares no code with it.

This is a thin ctypes wrapper around ``mci_oracle.c`` (direct O(N^2) DFT, Gaussian
elimination per residue, direct trigonometric sum on the output grid) plus two plain
NumPy helpers that state closed formulas of the paper:

* :func:`averaged_error` -- the exact phase-averaged squared error of Theorem 4.4
  (eq. averageerror),
* :func:`evaluate_band` -- the reconstruction's trigonometric sum (eq. DFTexpression) at
  arbitrary points, for sampled checks of outputs too long to evaluate in full, and
* :func:`psnr` -- peak signal-to-noise ratio of an image in [0, 1].

Multiplier kinds and output operators use the integer codes below; channel tables
(kind ``TABLE``) hold b_k(n) for n in [n1, n1 + M N).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

MULT_DERIV, MULT_HILBERT, MULT_TABLE = 0, 1, 2
OUT_IDENTITY, OUT_HILBERT, OUT_DERIV = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc_mci.so")
_lib = None


class OracleError(RuntimeError):
    """Raised when the oracle reports a singular system or invalid arguments."""

    def __init__(self, code: int, bad: int = 0):
        self.code = code
        self.bad = bad
        names = {1: "invalid argument", 2: "singular system", 5: "out of memory"}
        super().__init__(f"oracle error {code} ({names.get(code, '?')}), residue {bad}")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # build on first use: plain gcc, seconds

        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    pi = P(i32)
    pd = P(dbl)
    lib.orc_channel_dft.argtypes = [i32, i64, i64, i32, i64, pd, pd]
    lib.orc_inverse_tables.argtypes = [i32, i64, i64, pi, pi, pd, pd, pi]
    lib.orc_recover_band.argtypes = [i32, i64, i64, pi, pi, pd, i32, i32, i64, pd, pd, P(i64)]
    lib.orc_reconstruct_1d.argtypes = [i32, i64, i64, pi, pi, pd, i32, pi, pi, i64, i32, i32, i64, pd, pd, P(i64)]
    lib.orc_interp_function.argtypes = [i32, i64, i64, pi, pi, pd, i32, i64, pd, pd]
    lib.orc_sampling_series.argtypes = [i32, i64, i64, pi, pi, pd, pd, i64, pd, pd]
    lib.orc_upsample_2d.argtypes = [i64, i64, i64, i32, i32, pd, pd]
    lib.orc_num_threads.argtypes = []
    for name in ("orc_channel_dft", "orc_inverse_tables", "orc_recover_band", "orc_reconstruct_1d",
                 "orc_interp_function", "orc_sampling_series", "orc_upsample_2d", "orc_num_threads"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def default_n1(mu: int) -> int:
    """Default band start -floor((mu - 1) / 2): the symmetric band [-N, N] of the
    paper's examples for odd mu, and Ex. 3.10's [-N, N + 1] for even mu."""
    return -((mu - 1) // 2)


@dataclass
class Channels:
    """M channels with multipliers b_k (eq. sysfunction) on the band [n1, n1 + M N)."""

    N: int
    kinds: Sequence[int]
    orders: Sequence[int] = ()
    n1: Optional[int] = None
    tables: Optional[np.ndarray] = None  # complex [M][mu] for MULT_TABLE channels
    _k: np.ndarray = field(init=False, repr=False)
    _o: np.ndarray = field(init=False, repr=False)
    _t: Optional[np.ndarray] = field(init=False, repr=False)

    def __post_init__(self):
        M = len(self.kinds)
        orders = list(self.orders) if len(self.orders) else [0] * M
        if self.n1 is None:
            self.n1 = default_n1(M * self.N)
        self._k = np.ascontiguousarray(self.kinds, dtype=np.int32)
        self._o = np.ascontiguousarray(orders, dtype=np.int32)
        if self.tables is not None:
            t = np.asarray(self.tables, dtype=np.complex128).reshape(M, M * self.N)
            self._t = np.ascontiguousarray(t.view(np.float64))
        else:
            self._t = None

    @property
    def M(self) -> int:
        return len(self.kinds)

    @property
    def mu(self) -> int:
        return self.M * self.N

    def _args(self):
        pi = ctypes.POINTER(ctypes.c_int)
        pd = ctypes.POINTER(ctypes.c_double)
        t = self._t.ctypes.data_as(pd) if self._t is not None else ctypes.cast(None, pd)
        return (self.M, self.N, self.n1, self._k.ctypes.data_as(pi), self._o.ctypes.data_as(pi), t)

    def multiplier(self, k: int, n: np.ndarray) -> np.ndarray:
        """b_k(n) evaluated in NumPy (used by the tests to synthesise channels)."""
        n = np.asarray(n)
        kind = self.kinds[k]
        if kind == MULT_DERIV:
            return (1j * n.astype(np.float64)) ** int(self._o[k])
        if kind == MULT_HILBERT:
            return -1j * np.sign(n).astype(np.float64)
        tab = np.asarray(self.tables).reshape(self.M, self.mu)[k]
        off = n - self.n1
        out = np.zeros(n.shape, dtype=np.complex128)
        ok = (off >= 0) & (off < self.mu)
        out[ok] = tab[off[ok]]
        return out


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, bad: int = 0):
    if rc != 0:
        raise OracleError(rc, bad)


def channel_dft(g: np.ndarray, N: int, n1: int) -> np.ndarray:
    """d_m(n1 + i), i in [0, N) for samples g[..., M, N] (real or complex)."""
    real = not np.iscomplexobj(g)
    g = np.ascontiguousarray(g, dtype=np.float64 if real else np.complex128)
    shp = g.shape
    M = shp[-2]
    batch = int(np.prod(shp[:-2])) if len(shp) > 2 else 1
    out = np.zeros(shp, dtype=np.complex128)
    gv = g if real else g.view(np.float64)
    _check(_load().orc_channel_dft(M, N, n1, int(real), batch, _pd(gv), _pd(out.view(np.float64))))
    return out


def inverse_tables(ch: Channels):
    """(Q, singular) with Q[i] = H_n^{-1} for n = n1 + i (eq. defH), Q[i][m][k] = q_mk(n)."""
    q = np.zeros((ch.N, ch.M, ch.M), dtype=np.complex128)
    fl = np.zeros(ch.N, dtype=np.int32)
    _check(_load().orc_inverse_tables(*ch._args(), _pd(q.view(np.float64)),
                                      fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return q, fl.astype(bool)


def recover_band(ch: Channels, g: np.ndarray, allow_singular_zero: bool = False) -> np.ndarray:
    """Recovered coefficients a(n1 + i), i in [0, mu), for samples g[batch?, M, N]."""
    real = not np.iscomplexobj(g)
    g = np.ascontiguousarray(g, dtype=np.float64 if real else np.complex128)
    squeeze = g.ndim == 2
    if squeeze:
        g = g[None]
    batch = g.shape[0]
    out = np.zeros((batch, ch.mu), dtype=np.complex128)
    bad = ctypes.c_int64(0)
    rc = _load().orc_recover_band(*ch._args(), int(real), int(allow_singular_zero), batch,
                                  _pd(g if real else g.view(np.float64)), _pd(out.view(np.float64)),
                                  ctypes.byref(bad))
    _check(rc, bad.value)
    return out[0] if squeeze else out


def reconstruct_1d(ch: Channels, g: np.ndarray, n_out: int, ops: Sequence[int] = (OUT_IDENTITY,),
                   op_orders: Sequence[int] = (), allow_singular_zero: bool = False) -> np.ndarray:
    """Reconstruction on t_j = 2 pi j / n_out: out[batch?, n_ops, n_out].

    Real samples give Re of the reconstruction; complex samples give the complex
    reconstruction."""
    real = not np.iscomplexobj(g)
    g = np.ascontiguousarray(g, dtype=np.float64 if real else np.complex128)
    squeeze = g.ndim == 2
    if squeeze:
        g = g[None]
    batch = g.shape[0]
    if g.shape[1:] != (ch.M, ch.N):
        raise ValueError(f"samples must be [batch][{ch.M}][{ch.N}], got {g.shape}")
    n_ops = len(ops)
    op_orders = list(op_orders) if len(op_orders) else [0] * n_ops
    ops_a = np.ascontiguousarray(ops, dtype=np.int32)
    ord_a = np.ascontiguousarray(op_orders, dtype=np.int32)
    out = np.zeros((batch, n_ops, n_out), dtype=np.float64 if real else np.complex128)
    bad = ctypes.c_int64(0)
    pi = ctypes.POINTER(ctypes.c_int)
    rc = _load().orc_reconstruct_1d(*ch._args(), n_ops, ops_a.ctypes.data_as(pi), ord_a.ctypes.data_as(pi),
                                    n_out, int(real), int(allow_singular_zero), batch,
                                    _pd(g if real else g.view(np.float64)),
                                    _pd(out if real else out.view(np.float64)), ctypes.byref(bad))
    _check(rc, bad.value)
    return out[0] if squeeze else out


def interp_function(ch: Channels, m: int, t: np.ndarray) -> np.ndarray:
    """y_m(t) of eq. ym (0-based channel m) at real points t."""
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.zeros(t.size, dtype=np.complex128)
    _check(_load().orc_interp_function(*ch._args(), m, t.size, _pd(t), _pd(out.view(np.float64))))
    return out


def sampling_series(ch: Channels, g: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Theorem 3.3's sampling series (eq. drictexpression) at real points t."""
    g = np.ascontiguousarray(g, dtype=np.complex128).reshape(ch.M, ch.N)
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.zeros(t.size, dtype=np.complex128)
    _check(_load().orc_sampling_series(*ch._args(), _pd(g.view(np.float64)), t.size, _pd(t),
                                       _pd(out.view(np.float64))))
    return out


def upsample_2d(x: np.ndarray, s: int, M: int = 2) -> np.ndarray:
    """Separable rows-then-columns MCI upsampling by s with channels {x, Dx} (M = 2) or
    {x, Dx, D2x} (M = 3, the setting of Section 5.2's experiments), D and D2 the three-point
    centred first and second differences in t-units."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    squeeze = x.ndim == 2
    if squeeze:
        x = x[None]
    B, h, w = x.shape
    y = np.zeros((B, s * h, s * w), dtype=np.float64)
    _check(_load().orc_upsample_2d(B, h, w, s, M, _pd(x), _pd(y)))
    return y[0] if squeeze else y


def averaged_error(ch: Channels, coeff_n: np.ndarray, coeff_a: np.ndarray) -> float:
    """Exact phase-averaged error epsilon(f, N) of Theorem 4.4 (eq. averageerror).

    ``coeff_n``/``coeff_a`` list the (finitely many) nonzero Fourier coefficients a(n)
    of f.  With blocks I_k = [n1 + (k-1) N, n1 + k N - 1] (k 1-based) and r_m from
    eq. defrm,

      eps^2 = sum_{n not in band} |a(n)|^2
            + sum_{k not in 1..M} sum_{n in I_k} |a(n)|^2
                  * sum_{l=1..M} | sum_m r_m(n + (l - k) N) b_m(n) |^2 .
    """
    q, sing = inverse_tables(ch)
    if sing.any():
        raise OracleError(2)
    M, N, n1 = ch.M, ch.N, ch.n1
    n = np.asarray(coeff_n, dtype=np.int64)
    a2 = np.abs(np.asarray(coeff_a)) ** 2
    inband = (n >= n1) & (n < n1 + ch.mu)
    eps2 = float(a2[~inband].sum())
    k = np.floor_divide(n - n1, N) + 1          # 1-based block index
    res = np.mod(n - n1, N)                      # residue offset inside the block
    outside = ~inband
    bm = np.stack([ch.multiplier(m, n) for m in range(M)])  # [M][len(n)]
    for l in range(1, M + 1):
        # n + (l - k) N lies in block I_l at the same residue: r_m there is q_{m, l-1}(n1 + res)
        s = np.zeros(n.size, dtype=np.complex128)
        for m in range(M):
            s += q[res, m, l - 1] * bm[m]
        eps2 += float((a2[outside] * np.abs(s[outside]) ** 2).sum())
    del k
    return float(np.sqrt(eps2))


def evaluate_band(a: np.ndarray, n1: int, t: np.ndarray, op: int = OUT_IDENTITY, order: int = 0,
                  real: bool = True) -> np.ndarray:
    """sum_n o(n) a(n) e^{i n t} over the band n = n1 .. n1 + len(a) - 1 at real points t
    (eq. DFTexpression with the output operator of the closing paragraph of Section 3);
    the real part in real mode.  Direct sum, 64 points at a time."""
    a = np.asarray(a, dtype=np.complex128).ravel()
    n = np.arange(n1, n1 + a.size, dtype=np.float64)
    if op == OUT_IDENTITY:
        o = np.ones_like(n, dtype=np.complex128)
    elif op == OUT_HILBERT:
        o = -1j * np.sign(n)
    else:
        o = (1j * n) ** int(order)
    c = a * o
    t = np.asarray(t, dtype=np.float64).ravel()
    out = np.empty(t.size, dtype=np.complex128)
    for s0 in range(0, t.size, 64):
        tt = t[s0:s0 + 64]
        out[s0:s0 + 64] = np.exp(1j * np.outer(tt, n)) @ c
    return out.real if real else out


def psnr(img: np.ndarray, ref: np.ndarray, clip: bool = True) -> float:
    """10 log10(1 / MSE) for images with peak value 1.0 (optionally clipped to [0, 1])."""
    x = np.clip(img, 0.0, 1.0) if clip else img
    mse = float(np.mean((np.asarray(x, dtype=np.float64) - ref) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


# ------------------------------------------------------------------ residual CNN refiner
CNN_SLICES = {}
_o = 0
for _name, _n in (("W1", 32 * 27), ("b1", 32), ("W2", 32 * 288), ("b2", 32), ("W3", 32 * 288), ("b3", 32),
                  ("W4", 3 * 288), ("b4", 3)):
    CNN_SLICES[_name] = slice(_o, _o + _n)
    _o += _n
CNN_NPARAM = _o


def _cnn_lib():
    lib = _load()
    if not hasattr(lib, "_cnn_ready"):
        P = ctypes.POINTER
        pd = P(ctypes.c_double)
        lib.orc_cnn_forward.argtypes = [pd, ctypes.c_int64, ctypes.c_int, ctypes.c_int, pd, pd, ctypes.c_int]
        lib.orc_cnn_grad.argtypes = [pd, ctypes.c_int64, ctypes.c_int, ctypes.c_int, pd, pd, pd, pd, ctypes.c_int]
        lib.orc_cnn_forward.restype = ctypes.c_int
        lib.orc_cnn_grad.restype = ctypes.c_int
        lib.orc_bf16_round.argtypes = [ctypes.c_double]
        lib.orc_bf16_round.restype = ctypes.c_double
        lib._cnn_ready = True
    return lib


def bf16_round(x: float) -> float:
    """x rounded to the nearest BF16 value, ties to even (the rounding of ``bf16=True``)."""
    return float(_cnn_lib().orc_bf16_round(float(x)))


def cnn_forward(params: np.ndarray, u: np.ndarray, bf16: bool = False) -> np.ndarray:
    """y = u + CNN(u) for images u [B][3][H][W] (FP64, zero padding).  With ``bf16`` the
    weights, the network input and the hidden activations are rounded to BF16 where a BF16
    implementation stores them; the arithmetic stays FP64."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    assert p.size == CNN_NPARAM
    u = np.ascontiguousarray(u, dtype=np.float64)
    B, c, H, W = u.shape
    y = np.empty_like(u)
    _check(_cnn_lib().orc_cnn_forward(_pd(p), B, H, W, _pd(u), _pd(y), int(bool(bf16))))
    return y


def cnn_grad(params: np.ndarray, u: np.ndarray, hr: np.ndarray, bf16: bool = False):
    """(loss, grad): loss = mean((u + CNN(u) - hr)^2), grad = dloss/dparams (FP64).  With
    ``bf16`` the stored operands of the forward pass and the back-propagated gradients (the
    output gradient and each activation gradient after its ReLU mask) are rounded to BF16."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    hr = np.ascontiguousarray(hr, dtype=np.float64)
    B, c, H, W = u.shape
    g = np.zeros(CNN_NPARAM)
    loss = ctypes.c_double(0.0)
    _check(_cnn_lib().orc_cnn_grad(_pd(p), B, H, W, _pd(u), _pd(hr), _pd(g), ctypes.byref(loss), int(bool(bf16))))
    return loss.value, g


def omega(ch: Channels) -> np.ndarray:
    """Omega_m(L) = sup over the band of |r_m|^2 (the definition after Theorem 4.4); by
    eq. defrm r_m takes the values q_mk(n) of the inverse tables, k over the blocks and n
    over I_1, so Omega_m is the largest |q_mk(n)|^2.  Returns Omega_1..Omega_M."""
    q, sing = inverse_tables(ch)
    if sing.any():
        raise OracleError(2)
    return (np.abs(q) ** 2).max(axis=(0, 2))


def error_bound(ch: Channels, coeff_n: np.ndarray, coeff_a: np.ndarray) -> float:
    """The bound of eq. errorestimate on epsilon(f, N) (its square root):

      eps^2 <= sum_{n not in band} |a(n)|^2
             + M (sum_k Omega_k) sum_{n not in band} sum_m |a(n) b_m(n)|^2 .

    Cauchy-Schwarz on each |sum_m r_m b_m|^2 of eq. averageerror gives the factor
    sum_m sup |r_m|^2 = sum_m Omega_m once per l = 1..M.  The printed bound squares Omega_k,
    which the definition already makes a square; read literally that is no bound where
    Omega_k < 1 (derivative channels), so Omega_k enters once here."""
    om = omega(ch)
    n = np.asarray(coeff_n, dtype=np.int64)
    a2 = np.abs(np.asarray(coeff_a)) ** 2
    outside = ~((n >= ch.n1) & (n < ch.n1 + ch.mu))
    b2 = sum(np.abs(ch.multiplier(m, n)) ** 2 for m in range(ch.M))
    s1 = float(a2[outside].sum())
    s2 = float((a2[outside] * b2[outside]).sum())
    return float(np.sqrt(s1 + ch.M * float(om.sum()) * s2))
