"""Seeded 1-D signals and their channel samples.

Every signal is given by finitely many Fourier coefficients a(n) (eq. function), so
its channel samples g_m(t_p), t_p = 2 pi p / N, are exact finite sums.  They are
formed by folding b_m(n) a(n) modulo N and one FP64 inverse DFT of length N (NumPy's
pocketfft), which is the definition of the samples written as a library call.
"""
from __future__ import annotations

from typing import Callable, Sequence, Tuple

import numpy as np

Multiplier = Callable[[np.ndarray], np.ndarray]


def deriv_multiplier(order: int) -> Multiplier:
    """b(n) = (i n)^order: the order-th derivative channel."""
    return lambda n: (1j * np.asarray(n, dtype=np.float64)) ** order


def hilbert_multiplier() -> Multiplier:
    """b(n) = -i sgn n: the circular Hilbert transform channel."""
    return lambda n: -1j * np.sign(np.asarray(n)).astype(np.float64)


def sample_channels(n: np.ndarray, a: np.ndarray, mults: Sequence[Multiplier], N: int,
                    real: bool = False) -> np.ndarray:
    """g[m][p] = sum_n b_m(n) a(n) e^{2 pi i n p / N} for p in [0, N).

    ``n``/``a``: coefficient indices and values (1-D).  Returns complex [M][N], or its
    real part when ``real`` (use for real signals with real-valued channels)."""
    n = np.asarray(n, dtype=np.int64)
    a = np.asarray(a, dtype=np.complex128)
    out = np.empty((len(mults), N), dtype=np.complex128)
    k = np.mod(n, N)
    for m, b in enumerate(mults):
        folded = np.zeros(N, dtype=np.complex128)
        np.add.at(folded, k, b(n) * a)
        out[m] = np.fft.ifft(folded) * N
    return out.real.copy() if real else out


def trig_poly_real(seed: int, degree: int) -> Tuple[np.ndarray, np.ndarray]:
    """Real trigonometric polynomial alpha_0 + sum_{n=1}^{degree} alpha_n cos nt + beta_n sin nt,
    alpha, beta ~ N(0, 1).  Returns (n, a(n)) for n in [-degree, degree]."""
    rng = np.random.default_rng(seed)
    alpha = rng.standard_normal(degree + 1)
    beta = rng.standard_normal(degree + 1)
    n = np.arange(-degree, degree + 1)
    a = np.zeros(n.size, dtype=np.complex128)
    pos = np.arange(1, degree + 1)
    a[degree + pos] = 0.5 * (alpha[pos] - 1j * beta[pos])
    a[degree - pos] = 0.5 * (alpha[pos] + 1j * beta[pos])
    a[degree] = alpha[0]
    return n, a


def random_bandlimited(seed: int, n_lo: int, n_hi: int) -> Tuple[np.ndarray, np.ndarray]:
    """Complex coefficients a(n) ~ CN(0, 1) on [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    n = np.arange(n_lo, n_hi + 1)
    a = (rng.standard_normal(n.size) + 1j * rng.standard_normal(n.size)) / np.sqrt(2.0)
    return n, a


def single_signal_fp64(seed: int = 1, degree: int = 127, N: int = 128):
    """One real trigonometric polynomial of degree `degree` (L = 2 degree + 2 band slots)
    sampled with channels {f, f'} at N points each.  Returns (g[2][N] f64, n, a)."""
    n, a = trig_poly_real(seed, degree)
    g = sample_channels(n, a, [deriv_multiplier(0), deriv_multiplier(1)], N, real=True)
    return g, n, a


def smooth_noisy_spectrum(rng: np.random.Generator, n_max: int, decay: float = 0.01,
                          noise: float = 1e-3) -> Tuple[np.ndarray, np.ndarray]:
    """Hermitian spectrum c_n = e^{-decay |n|} z_n + noise w_n on [-n_max, n_max],
    z_n, w_n ~ CN(0, 1) for n > 0 (real for n = 0), c_{-n} = conj(c_n)."""
    z = (rng.standard_normal(n_max) + 1j * rng.standard_normal(n_max)) / np.sqrt(2.0)
    w = (rng.standard_normal(n_max) + 1j * rng.standard_normal(n_max)) / np.sqrt(2.0)
    z0, w0 = rng.standard_normal(2)
    pos = np.arange(1, n_max + 1)
    cpos = np.exp(-decay * pos) * z + noise * w
    n = np.arange(-n_max, n_max + 1)
    c = np.empty(n.size, dtype=np.complex128)
    c[n_max + 1:] = cpos
    c[:n_max] = np.conj(cpos[::-1])
    c[n_max] = z0 + noise * w0
    return n, c


def smooth_noisy_batch(first: int, count: int, M: int, N: int, n_max: int, seed_base: int = 2_000_000,
                       dtype=np.float32, deriv_scale: float = 1.0) -> np.ndarray:
    """Samples [count][M][N] of signals first .. first+count-1.

    Signal s draws its spectrum from ``numpy.random.default_rng(seed_base + s)``
    (:func:`smooth_noisy_spectrum`) and is sampled with the derivative channels
    b_m(n) = (i n / deriv_scale)^m, m = 0 .. M-1, at t_p = 2 pi p / N (deriv_scale = N
    keeps every channel within a small factor of the signal's own size, which FP16
    storage needs).  The FP64 samples are rounded once to ``dtype``."""
    out = np.empty((count, M, N), dtype=dtype)
    n = np.arange(-n_max, n_max + 1)
    k = np.mod(n, N)
    # fold c_n (i n)^m modulo N with a dense reshape: pad the index range to a multiple of N
    lo = -n_max - np.mod(-n_max, N)          # first multiple of N at or below -n_max
    span = ((n_max - lo) // N + 1) * N
    pad_start = -n_max - lo
    powers = [(1j * n.astype(np.float64) / deriv_scale) ** m for m in range(M)]
    for s in range(count):
        rng = np.random.default_rng(seed_base + first + s)
        _, c = smooth_noisy_spectrum(rng, n_max)
        for m in range(M):
            buf = np.zeros(span, dtype=np.complex128)
            buf[pad_start:pad_start + n.size] = powers[m] * c
            folded = buf.reshape(-1, N).sum(axis=0)   # index r in row q is lo + qN + r == r (mod N) as lo % N == 0
            out[s, m] = (np.fft.ifft(folded) * N).real
    del k
    return out


# ---------------------------------------------------------------- the test signal of Section 5.1
def phi_closed(z: np.ndarray) -> np.ndarray:
    """The rational function phi of Section 5.1 (analytic in the closed unit disc)."""
    return (0.08 * z**2 + 0.06 * z**10) / ((1.3 - z) * (1.5 - z)) + \
           (0.05 * z**3 + 0.09 * z**10) / ((1.2 + z) * (1.3 + z))


def _taylor(P, Q, nmax):
    """Taylor coefficients of P(z)/Q(z) at 0 by the recurrence sum_j Q_j c_{n-j} = P_n."""
    c = np.zeros(nmax + 1)
    for n in range(nmax + 1):
        s = P[n] if n < len(P) else 0.0
        for j in range(1, len(Q)):
            if n - j >= 0:
                s -= Q[j] * c[n - j]
        c[n] = s / Q[0]
    return c


def phi_coeffs(nmax: int = 700) -> np.ndarray:
    """Power-series coefficients c_0 .. c_nmax of phi (its poles lie at |z| >= 1.2, so the
    terms past n = 700 are below 1e-55 of the leading ones)."""
    P1 = np.zeros(11); P1[2] = 0.08; P1[10] = 0.06
    P2 = np.zeros(11); P2[3] = 0.05; P2[10] = 0.09
    # (1.3 - z)(1.5 - z) = 1.95 - 2.8 z + z^2 ; (1.2 + z)(1.3 + z) = 1.56 + 2.5 z + z^2
    return _taylor(P1, [1.95, -2.8, 1.0], nmax) + _taylor(P2, [1.56, 2.5, 1.0], nmax)


def phi_samples(kind: str, t: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Samples at t of f = Re phi(e^{it}) (kind 'f'), its Hilbert transform Im phi(e^{it})
    ('H'), and the derivatives f' ('d1') and f'' ('d2'), from the power series c of phi."""
    if kind == "f":
        return phi_closed(np.exp(1j * t)).real
    if kind == "H":
        return phi_closed(np.exp(1j * t)).imag
    order = {"d1": 1, "d2": 2}[kind]
    n = np.arange(c.size)
    return (((1j * n) ** order) * c[None, :] * np.exp(1j * np.outer(t, n))).sum(1).real
