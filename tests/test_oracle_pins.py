"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with something
else -- values the paper prints (Table 1), closed forms the paper derives (Examples
3.5-3.10), theorems (3.3 exact recovery, 4.1 consistency, 4.4 averaged error,
Lemma 4.2), library routines the method reduces to (NumPy zero-padded FFT
interpolation, SciPy's discrete Hilbert transform), or the independent sampling-series
route.  A dropped term, a sign error, a transposed solve or a wrong alias index in the
oracle fails at least one of them.
"""
import os

import numpy as np
import pytest
import scipy.signal

from oracle import oracle as O
from synth import signals as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- test signal of Section 5.1
_phi = S.phi_closed
_phi_coeffs = S.phi_coeffs
_phi_channel = S.phi_samples


def test_phi_series_matches_closed_form():
    c = _phi_coeffs()
    n = np.arange(c.size)
    t = np.linspace(0.0, 2 * np.pi, 41)
    ser = (c[None, :] * np.exp(1j * np.outer(t, n))).sum(1)
    assert np.abs(ser - _phi(np.exp(1j * t))).max() < 1e-13


@pytest.mark.parametrize("N,n1", [(12, -17), (13, 5), (1, 0), (7, -3)])
@pytest.mark.parametrize("real", [True, False])
def test_channel_dft_equals_numpy_fft(N, n1, real):
    """Lemma 3.1's d_m(n) = (1/N) sum_p g_m[p] e^{-2 pi i n p / N} for n = n1 + i: NumPy's FFT
    divided by N, read at n mod N, for every (signal, channel) of a batch; and a single
    exponential e^{i k t_p} has d(n) = 1 exactly where n = k mod N."""
    rng = np.random.default_rng(N + 100 * real)
    B, M = 3, 4
    g = rng.standard_normal((B, M, N))
    if not real:
        g = g + 1j * rng.standard_normal((B, M, N))
    d = O.channel_dft(g, N, n1)
    idx = np.mod(n1 + np.arange(N), N)
    want = np.fft.fft(g, axis=-1)[..., idx] / N
    assert d.shape == (B, M, N)
    assert np.abs(d - want).max() <= 1e-13
    k = 5
    e = np.exp(1j * k * 2 * np.pi * np.arange(N) / N)[None, None]
    d1 = O.channel_dft(e, N, n1)[0, 0]
    hit = np.mod(n1 + np.arange(N) - k, N) == 0
    assert np.abs(d1[hit] - 1).max() <= 1e-13 and np.abs(d1[~hit]).max(initial=0.0) <= 1e-13


def _load_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows.append((int(v[0]), int(v[1]), int(v[2]), int(v[3]), int(v[4]), float(v[5]), float(v[6])))
    return rows


def _sig4(x):
    return float(f"{x:.4g}")


def test_table1_reproduces():
    """Table 1 (Section 5.1): 31 of the 32 printed RMS errors reproduce to 4 significant
    digits when real data give Re of the reconstruction and delta_2 applies the Hilbert
    multiplier to the spectrum recovered from the same channels.  The one cell that does
    not (mu = 96, 48 f + 48 Hf, delta_2 printed 0.3836e-2) recomputes to 0.3869e-2
    under the reading that reproduces all the others, so it is taken as a misprint."""
    c = _phi_coeffs()
    tg = 2 * np.pi * np.arange(2048) / 2048
    F, HF = _phi_channel("f", tg, c), _phi_channel("H", tg, c)
    checked = 0
    for mu, nf, nh, nd1, nd2, d1, d2 in _load_table1():
        if nh:
            kinds, orders, names = [O.MULT_DERIV, O.MULT_HILBERT], [0, 0], ["f", "H"]
        elif nd1:
            kinds, orders, names = [O.MULT_DERIV] * 3, [0, 1, 2], ["f", "d1", "d2"]
        else:
            kinds, orders, names = [O.MULT_DERIV], [0], ["f"]
        M = len(kinds)
        N = mu // M
        assert N == nf
        ch = O.Channels(N=N, kinds=kinds, orders=orders)
        tp = 2 * np.pi * np.arange(N) / N
        g = np.stack([_phi_channel(k, tp, c) for k in names])
        y = O.reconstruct_1d(ch, g, 2048, ops=[O.OUT_IDENTITY, O.OUT_HILBERT])
        e1 = np.linalg.norm(F - y[0]) / np.linalg.norm(F)
        e2 = np.linalg.norm(HF - y[1]) / np.linalg.norm(HF)
        assert _sig4(e1) == pytest.approx(d1, rel=1e-9), (mu, names, e1, d1)
        if mu == 96 and nh:
            assert _sig4(e2) == pytest.approx(0.003869, rel=1e-9)
            assert abs(e2 - d2) / d2 > 5e-3   # the printed value is not reproduced
        else:
            assert _sig4(e2) == pytest.approx(d2, rel=1e-9), (mu, names, e2, d2)
        checked += 1
    assert checked == 16


def test_table1_reading_alternatives_fail():
    """The two readings the pins rely on are forced: the complex reconstruction (no Re)
    and running MCI on Hf's own channels both miss the printed values."""
    c = _phi_coeffs()
    tg = 2 * np.pi * np.arange(2048) / 2048
    F, HF = _phi_channel("f", tg, c), _phi_channel("H", tg, c)
    # mu = 24, 24 samples of f: complex reconstruction gives 1.1316, not 1.067
    ch = O.Channels(N=24, kinds=[O.MULT_DERIV], orders=[0])
    tp = 2 * np.pi * np.arange(24) / 24
    yc = O.reconstruct_1d(ch, _phi_channel("f", tp, c)[None].astype(complex), 2048)[0]
    assert abs(np.linalg.norm(F - yc) / np.linalg.norm(F) - 1.067) > 0.05
    # mu = 32, 16 f + 16 Hf: MCI applied to Hf's channels (Hf, H Hf = -f + a0) gives 0.6795, not 0.7532
    ch2 = O.Channels(N=16, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0])
    tp = 2 * np.pi * np.arange(16) / 16
    a0 = 0.0  # phi(0) = 0, so f has zero mean
    g_alt = np.stack([_phi_channel("H", tp, c), -_phi_channel("f", tp, c) + a0])
    y_alt = O.reconstruct_1d(ch2, g_alt, 2048)[0]
    assert abs(np.linalg.norm(HF - y_alt) / np.linalg.norm(HF) - 0.7532) > 0.05


# ---------------------------------------------------------------- Theorem 3.3: exact recovery
CHANNEL_SETS = [
    ("f", [O.MULT_DERIV], [0]),
    ("f,f'", [O.MULT_DERIV] * 2, [0, 1]),
    ("f,f',f''", [O.MULT_DERIV] * 3, [0, 1, 2]),
    ("f..f'''", [O.MULT_DERIV] * 4, [0, 1, 2, 3]),
    ("f,Hf", [O.MULT_DERIV, O.MULT_HILBERT], [0, 0]),
    ("f',f''", [O.MULT_DERIV] * 2, [1, 2]),
]


def _random_table_channels(M, N, seed):
    rng = np.random.default_rng(seed)
    tab = rng.standard_normal((M, M * N)) + 1j * rng.standard_normal((M, M * N))
    return O.Channels(N=N, kinds=[O.MULT_TABLE] * M, orders=[0] * M, tables=tab)


@pytest.mark.parametrize("name,kinds,orders", CHANNEL_SETS)
@pytest.mark.parametrize("N,n_out", [(9, 64), (8, 40), (16, 21)])
def test_exact_recovery_bandlimited(name, kinds, orders, N, n_out):
    """f in B_N is recovered exactly at every output point (Theorem 3.3), including
    output grids coarser than the band (n_out = 21 < mu folds)."""
    ch = O.Channels(N=N, kinds=kinds, orders=orders)
    if name == "f',f''":      # b_1(0) = 0 makes H_n singular at n = 0 unless 0 is avoided
        ch = O.Channels(N=N, kinds=kinds, orders=orders, n1=1)
    n, a = S.random_bandlimited(seed=11 + N, n_lo=ch.n1, n_hi=ch.n1 + ch.mu - 1)
    g = S.sample_channels(n, a, [lambda k, m=m: ch.multiplier(m, k) for m in range(ch.M)], N)
    y = O.reconstruct_1d(ch, g, n_out, ops=[O.OUT_IDENTITY, O.OUT_HILBERT, O.OUT_DERIV], op_orders=[0, 0, 1])
    tj = 2 * np.pi * np.arange(n_out) / n_out
    E = np.exp(1j * np.outer(tj, n))
    f = E @ a
    Hf = E @ (-1j * np.sign(n) * a)
    df = E @ (1j * n * a)
    for got, want in ((y[0], f), (y[1], Hf), (y[2], df)):
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


def test_exact_recovery_random_multipliers():
    for M in (2, 3, 4):
        ch = _random_table_channels(M, 7, seed=M)
        n, a = S.random_bandlimited(seed=100 + M, n_lo=ch.n1, n_hi=ch.n1 + ch.mu - 1)
        g = S.sample_channels(n, a, [lambda k, m=m: ch.multiplier(m, k) for m in range(M)], ch.N)
        y = O.reconstruct_1d(ch, g, 50)[0]
        f = np.exp(1j * np.outer(2 * np.pi * np.arange(50) / 50, n)) @ a
        assert np.linalg.norm(y - f) <= 1e-11 * np.linalg.norm(f)


def test_exact_recovery_real_c1_shape():
    """The single-signal FP64 workload: a real trigonometric polynomial of degree 127,
    channels f and f' with 128 samples each, band [-127, 128], 4096 output points."""
    g, n, a = S.single_signal_fp64(seed=1, degree=127, N=128)
    ch = O.Channels(N=128, kinds=[O.MULT_DERIV] * 2, orders=[0, 1])
    assert ch.n1 == -127
    y = O.reconstruct_1d(ch, g, 4096, ops=[O.OUT_IDENTITY, O.OUT_HILBERT])
    tj = 2 * np.pi * np.arange(4096) / 4096
    E = np.exp(1j * np.outer(tj, n))
    f = (E @ a).real
    Hf = (E @ (-1j * np.sign(n) * a)).real
    assert np.linalg.norm(y[0] - f) <= 1e-12 * np.linalg.norm(f)
    assert np.linalg.norm(y[1] - Hf) <= 1e-12 * np.linalg.norm(Hf)


# ---------------------------------------------------------------- Theorem 4.1: consistency
def test_consistency_non_bandlimited_real():
    """(T f * h_m)(t_p) = g_m(t_p) for a non-bandlimited f (Theorem 4.1), checked through
    the real-mode output with derivative output operators on the sample grid."""
    rng = np.random.default_rng(5)
    n, c = S.smooth_noisy_spectrum(rng, n_max=60, decay=0.05, noise=1e-2)
    N = 11
    g = S.sample_channels(n, c, [S.deriv_multiplier(m) for m in range(3)], N, real=True)
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    for n_out, step in ((N, 1), (3 * N, 3)):
        y = O.reconstruct_1d(ch, g, n_out, ops=[O.OUT_IDENTITY, O.OUT_DERIV, O.OUT_DERIV], op_orders=[0, 1, 2])
        for m in range(3):
            assert np.abs(y[m, ::step] - g[m]).max() <= 1e-10 * np.abs(g[m]).max()


def test_consistency_non_bandlimited_complex_hilbert():
    rng = np.random.default_rng(6)
    n = np.arange(-40, 41)
    a = (rng.standard_normal(n.size) + 1j * rng.standard_normal(n.size)) * np.exp(-0.03 * np.abs(n))
    ch = O.Channels(N=10, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0])
    mults = [S.deriv_multiplier(0), lambda k: -1j * np.sign(k)]
    g = S.sample_channels(n, a, mults, ch.N)
    band = O.recover_band(ch, g)
    nb = np.arange(ch.n1, ch.n1 + ch.mu)
    tp = 2 * np.pi * np.arange(ch.N) / ch.N
    for m in range(2):
        back = np.exp(1j * np.outer(tp, nb)) @ (band * mults[m](nb))
        assert np.abs(back - g[m]).max() <= 1e-12 * np.abs(g[m]).max()


# ---------------------------------------------------------------- closed-form inverses
def test_example_3_6_inverse_closed_form():
    """H_n^{-1} for {f, f', f''} printed in Example 3.6 (L = samples per channel)."""
    L = 7
    ch = O.Channels(N=L, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    q, sing = O.inverse_tables(ch)
    assert not sing.any()
    for i in range(L):
        n = ch.n1 + i
        want = np.array([
            [(2 * L**2 + 3 * L * n + n**2) / (2 * L**2), -n * (2 * L + n) / L**2, n * (L + n) / (2 * L**2)],
            [1j * (3 * L + 2 * n) / (2 * L**2), -2j * (L + n) / L**2, 1j * (L + 2 * n) / (2 * L**2)],
            [-1 / (2 * L**2), 1 / L**2, -1 / (2 * L**2)]])
        assert np.abs(q[i] - want).max() < 1e-14


def test_two_derivative_channels_inverse_closed_form():
    """{f, f'}: H_n = [[1, i n], [1, i (n + N)]], so H_n^{-1} = [[(n+N)/N, -n/N], [i/N, -i/N]]."""
    N = 128
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 2, orders=[0, 1])
    q, _ = O.inverse_tables(ch)
    n = ch.n1 + np.arange(N)
    want = np.empty((N, 2, 2), dtype=complex)
    want[:, 0, 0] = (n + N) / N
    want[:, 0, 1] = -n / N
    want[:, 1, 0] = 1j / N
    want[:, 1, 1] = -1j / N
    assert np.abs(q - want).max() < 1e-14


def test_example_3_10_inverse_and_erratum():
    """{f, Hf} on [-N', N'+1]: H_n^{-1} = [[1/2, 1/2], [-i/2, i/2]] for n < 0; at n = 0 the
    inverse is [[1, 0], [-i, i]] (the printed [[1, 0], [-i, 1]] does not invert H_0)."""
    Np = 6
    ch = O.Channels(N=Np + 1, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0])
    assert ch.n1 == -Np
    q, sing = O.inverse_tables(ch)
    assert not sing.any()
    for i in range(Np):
        assert np.abs(q[i] - np.array([[0.5, 0.5], [-0.5j, 0.5j]])).max() < 1e-15
    assert np.abs(q[Np] - np.array([[1, 0], [-1j, 1j]])).max() < 1e-15
    H0 = np.array([[1, 0], [1, -1j]])
    assert np.abs(np.array([[1, 0], [-1j, 1]]) @ H0 - np.eye(2)).max() > 0.5


def test_lemma_4_2_identities():
    """sum_m r_m(n) b_m(n) = 1 on the band and 0 for n1 - n2 a nonzero multiple of N
    (Lemma 4.2), for random multipliers."""
    for M in (2, 3, 4):
        ch = _random_table_channels(M, 5, seed=40 + M)
        q, _ = O.inverse_tables(ch)
        nb = np.arange(ch.n1, ch.n1 + ch.mu)
        r = np.zeros((M, ch.mu), dtype=complex)
        for i in range(ch.mu):
            r[:, i] = q[i % ch.N, :, i // ch.N]
        b = np.stack([ch.multiplier(m, nb) for m in range(M)])
        for i1 in range(ch.mu):
            for i2 in range(ch.mu):
                if (i1 - i2) % ch.N:
                    continue
                s = (r[:, i1] * b[:, i2]).sum()
                assert abs(s - (1.0 if i1 == i2 else 0.0)) < 1e-12


# ---------------------------------------------------------------- closed-form interpolation functions
def _grid_away_from_zero(k=97):
    t = np.linspace(0.05, 2 * np.pi - 0.05, k)
    return t


def test_example_3_5_dirichlet_kernel():
    Nh = 6
    ch = O.Channels(N=2 * Nh + 1, kinds=[O.MULT_DERIV], orders=[0])
    t = _grid_away_from_zero()
    want = np.sin((Nh + 0.5) * t) / np.sin(t / 2)
    assert np.abs(O.interp_function(ch, 0, t) - want).max() < 1e-12


def test_example_3_6_interpolation_functions():
    N0 = 3
    L = 2 * N0 + 1
    ch = O.Channels(N=L, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    assert ch.n1 == -(3 * N0 + 1)
    t = _grid_away_from_zero()
    s3 = np.sin((N0 + 0.5) * t) ** 3
    den = (2 * N0 + 1) ** 2
    y1 = s3 * (N0**2 + N0 + 1 - (N0 + 1) * N0 * np.cos(t)) / (den * np.sin(t / 2) ** 3)
    y2 = np.sin(t) * s3 / (den * np.sin(t / 2) ** 3)
    y3 = 2 * s3 / (den * np.sin(t / 2))
    for m, want in enumerate((y1, y2, y3)):
        assert np.abs(O.interp_function(ch, m, t) - want).max() < 1e-12


def test_example_3_7_hilbert_only_kernel_with_remark_3_4():
    """M = 1, b = -i sgn n: H_0 is singular; with q(0) = 0 (Remark 3.4) the kernel is
    y(t) = -2 csc(t/2) sin(Nt/2) sin((1+N)t/2)."""
    Nh = 5
    ch = O.Channels(N=2 * Nh + 1, kinds=[O.MULT_HILBERT], orders=[0])
    q, sing = O.inverse_tables(ch)
    assert sing[Nh] and sing.sum() == 1       # residue n = 0 only
    t = _grid_away_from_zero()
    want = -2 / np.sin(t / 2) * np.sin(Nh * t / 2) * np.sin((1 + Nh) * t / 2)
    assert np.abs(O.interp_function(ch, 0, t) - want).max() < 1e-12


def test_example_3_9_analytic_kernel():
    Nh = 7
    ch = O.Channels(N=Nh + 1, kinds=[O.MULT_DERIV], orders=[0], n1=0)
    t = _grid_away_from_zero()
    yr = np.cos(Nh * t / 2) * np.sin((1 + Nh) * t / 2) / np.sin(t / 2)
    yi = np.sin(Nh * t / 2) * np.sin((1 + Nh) * t / 2) / np.sin(t / 2)
    assert np.abs(O.interp_function(ch, 0, t) - (yr + 1j * yi)).max() < 1e-12


def test_example_3_10_kernels_and_erratum():
    Np = 6
    ch = O.Channels(N=Np + 1, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0])
    t = _grid_away_from_zero()
    y1 = (np.cos((Np + 1) * t) - np.cos(Np * t) + np.cos(t) - 1) / (2 * np.cos(t) - 2)
    tail = 1j * (np.exp(-1j * Np * t) - 1) * (np.exp(1j * (Np + 1) * t) - 1) / (2 * (np.exp(1j * t) - 1))
    y2_fixed = 1j * np.exp(1j * (Np + 1) * t) - 1j - tail
    y2_printed = np.exp(1j * (Np + 1) * t) - 1j - tail
    assert np.abs(O.interp_function(ch, 0, t) - y1).max() < 1e-12
    got2 = O.interp_function(ch, 1, t)
    assert np.abs(got2 - y2_fixed).max() < 1e-12
    assert np.abs(got2 - y2_printed).max() > 1.0


# ---------------------------------------------------------------- library special cases
@pytest.mark.parametrize("N", [33, 32])
def test_example_3_5_equals_fft_zero_padding(N):
    """M = 1, b = 1 is trigonometric interpolation: NumPy's zero-padded FFT interpolation
    (the Nyquist bin split in half for even N)."""
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N)
    n_out = 128
    X = np.fft.fft(x)
    Y = np.zeros(n_out, dtype=complex)
    if N % 2:
        h = (N - 1) // 2
        Y[:h + 1] = X[:h + 1]
        Y[-h:] = X[-h:]
    else:
        h = N // 2
        Y[:h] = X[:h]
        Y[-(h - 1):] = X[-(h - 1):]
        Y[h] = X[h] / 2
        Y[n_out - h] = X[h] / 2
    want = np.fft.ifft(Y).real * n_out / N
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV], orders=[0])
    got = O.reconstruct_1d(ch, x[None], n_out)[0]
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max() * 10


@pytest.mark.parametrize("N", [31, 64])
def test_remark_3_8_discrete_hilbert(N):
    """On the sample grid the Hilbert output equals the discrete Hilbert transform
    (imaginary part of scipy.signal.hilbert), odd and even N."""
    rng = np.random.default_rng(N + 3)
    x = rng.standard_normal(N)
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV], orders=[0])
    got = O.reconstruct_1d(ch, x[None], N, ops=[O.OUT_HILBERT])[0]
    want = scipy.signal.hilbert(x).imag
    assert np.abs(got - want).max() < 1e-13


def test_hilbert_pairs_cos_to_sin():
    """H cos(nt) = sin(nt) and H kills the mean (Section 2)."""
    N = 16
    t = 2 * np.pi * np.arange(N) / N
    f = 0.7 + np.cos(3 * t) + 0.5 * np.cos(7 * t) - 0.2 * np.sin(5 * t)
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV], orders=[0])
    tj = 2 * np.pi * np.arange(200) / 200
    got = O.reconstruct_1d(ch, f[None], 200, ops=[O.OUT_HILBERT])[0]
    want = np.sin(3 * tj) + 0.5 * np.sin(7 * tj) + 0.2 * np.cos(5 * tj)
    assert np.abs(got - want).max() < 1e-13


# ---------------------------------------------------------------- independent second route
@pytest.mark.parametrize("M", [1, 2, 3])
def test_main_route_equals_sampling_series(M):
    """The DFT -> solve -> trigonometric-sum route equals the sampling series of
    Theorem 3.3 (eq. drictexpression) for arbitrary (non-bandlimited) samples."""
    N = 5
    ch = _random_table_channels(M, N, seed=70 + M)
    rng = np.random.default_rng(80 + M)
    g = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    n_out = 23
    tj = 2 * np.pi * np.arange(n_out) / n_out
    main = O.reconstruct_1d(ch, g, n_out)[0]
    series = O.sampling_series(ch, g, tj)
    assert np.abs(main - series).max() < 1e-11 * np.abs(series).max()
    # derivative channels as well
    chd = O.Channels(N=N, kinds=[O.MULT_DERIV] * M, orders=list(range(M)))
    assert np.abs(O.reconstruct_1d(chd, g, n_out)[0] - O.sampling_series(chd, g, tj)).max() < 1e-11 * \
        np.abs(O.sampling_series(chd, g, tj)).max()


# ---------------------------------------------------------------- Theorem 4.4
@pytest.mark.parametrize("setup", ["deriv2", "deriv3", "hilbert2"])
def test_theorem_4_4_averaged_error(setup):
    """The phase-averaged squared error over tau in [0, 2 pi / N) equals eq. averageerror.
    The error is a trigonometric polynomial in tau of harmonic index below 16, so 16
    equispaced phases average it exactly."""
    N = 6
    if setup == "deriv2":
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 2, orders=[0, 1])
        mults = [S.deriv_multiplier(0), S.deriv_multiplier(1)]
    elif setup == "deriv3":
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
        mults = [S.deriv_multiplier(m) for m in range(3)]
    else:
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0])
        mults = [S.deriv_multiplier(0), lambda k: -1j * np.sign(k)]
    rng = np.random.default_rng(9)
    n = np.arange(ch.n1 - 2 * N, ch.n1 + ch.mu + 2 * N)
    a = (rng.standard_normal(n.size) + 1j * rng.standard_normal(n.size)) * np.exp(-0.05 * np.abs(n))
    inband = (n >= ch.n1) & (n < ch.n1 + ch.mu)
    K = 16
    vals = []
    for q in range(K):
        tau = 2 * np.pi * q / (N * K)
        at = a * np.exp(-1j * n * tau)
        g = S.sample_channels(n, at, mults, N)
        rec = O.recover_band(ch, g)
        vals.append(np.sum(np.abs(a[~inband]) ** 2) + np.sum(np.abs(at[inband] - rec) ** 2))
    eps_avg = np.sqrt(np.mean(vals))
    eps_formula = O.averaged_error(ch, n, a)
    assert eps_avg == pytest.approx(eps_formula, rel=1e-10)
    # and it vanishes for a bandlimited signal
    assert O.averaged_error(ch, n[inband], a[inband]) == 0.0


def test_omega_closed_forms():
    """Omega_m(L) = sup |r_m|^2 from the closed-form inverses: Example 3.6 ({f, f', f''}) and
    the two-derivative set, whose entries are read off H_n^{-1} over n in I_1; Example
    3.10's {f, Hf} has Omega = (1, 1) (entries 1/2 and, at n = 0, 1 and |-i| = 1)."""
    L = 9
    ch = O.Channels(N=L, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    n = ch.n1 + np.arange(L)
    rows = [np.stack([(2 * L**2 + 3 * L * n + n**2) / (2 * L**2), -n * (2 * L + n) / L**2, n * (L + n) / (2 * L**2)]),
            np.stack([(3 * L + 2 * n) / (2 * L**2), -2 * (L + n) / L**2, (L + 2 * n) / (2 * L**2)]),
            np.stack([np.full(L, -1 / (2 * L**2)), np.full(L, 1 / L**2), np.full(L, -1 / (2 * L**2))])]
    want = np.array([(np.abs(r) ** 2).max() for r in rows])
    assert np.allclose(O.omega(ch), want, rtol=1e-13, atol=0)
    N = 20
    ch2 = O.Channels(N=N, kinds=[O.MULT_DERIV] * 2, orders=[0, 1])
    n2 = ch2.n1 + np.arange(N)
    want2 = [max((((n2 + N) / N) ** 2).max(), ((n2 / N) ** 2).max()), 1 / N**2]
    assert np.allclose(O.omega(ch2), want2, rtol=1e-13, atol=0)
    ch3 = O.Channels(N=7, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0])
    assert np.allclose(O.omega(ch3), [1.0, 1.0], rtol=1e-14)


@pytest.mark.parametrize("setup", ["deriv2", "deriv3", "hilbert2", "plain"])
def test_theorem_4_4_error_bound(setup):
    """eq. errorestimate bounds eq. averageerror for random non-bandlimited spectra; both
    vanish for a bandlimited signal; with one plain channel (b = 1, r = 1, Omega = 1) the
    bound is attained: both equal 2 sum_{n outside the band} |a(n)|^2."""
    N = 10
    kinds, orders = {"deriv2": ([O.MULT_DERIV] * 2, [0, 1]), "deriv3": ([O.MULT_DERIV] * 3, [0, 1, 2]),
                     "hilbert2": ([O.MULT_DERIV, O.MULT_HILBERT], [0, 0]), "plain": ([O.MULT_DERIV], [0])}[setup]
    ch = O.Channels(N=N, kinds=kinds, orders=orders)
    rng = np.random.default_rng(len(setup))
    n = np.arange(ch.n1 - 4 * N, ch.n1 + ch.mu + 4 * N)
    inband = (n >= ch.n1) & (n < ch.n1 + ch.mu)
    for trial in range(20):
        a = (rng.standard_normal(n.size) + 1j * rng.standard_normal(n.size)) * \
            np.exp(-rng.uniform(0.01, 0.5) * np.abs(n))
        eps, bound = O.averaged_error(ch, n, a), O.error_bound(ch, n, a)
        assert bound >= eps * (1 - 1e-12), (trial, eps, bound)
        if setup == "plain":
            out2 = np.sum(np.abs(a[~inband]) ** 2)
            assert eps == pytest.approx(np.sqrt(2 * out2), rel=1e-12)
            assert bound == pytest.approx(np.sqrt(2 * out2), rel=1e-12)
    assert O.error_bound(ch, n[inband], a[inband]) == 0.0 and O.averaged_error(ch, n[inband], a[inband]) == 0.0


# ---------------------------------------------------------------- singular systems (Remark 3.4)
def test_hilbert_only_needs_remark_3_4():
    Nh = 6
    ch = O.Channels(N=2 * Nh + 1, kinds=[O.MULT_HILBERT], orders=[0])
    n, a = S.random_bandlimited(seed=3, n_lo=-Nh, n_hi=Nh)
    a[Nh] = 0.0                                         # a(0) = 0, as Example 3.7 requires
    g = S.sample_channels(n, a, [lambda k: -1j * np.sign(k)], ch.N)
    with pytest.raises(O.OracleError) as ei:
        O.reconstruct_1d(ch, g, 40)
    assert ei.value.code == 2 and ei.value.bad == 0
    y = O.reconstruct_1d(ch, g, 40, allow_singular_zero=True)[0]
    want = np.exp(1j * np.outer(2 * np.pi * np.arange(40) / 40, n)) @ a
    assert np.abs(y - want).max() < 1e-12


def test_band_not_straddling_zero_is_singular_for_hilbert_pair():
    ch = O.Channels(N=5, kinds=[O.MULT_DERIV, O.MULT_HILBERT], orders=[0, 0], n1=1)
    _, sing = O.inverse_tables(ch)
    assert sing.all()


# ---------------------------------------------------------------- 2-D separable upsampling
def test_2d_decimation_consistency():
    """out[s i, s j] = LR[i, j] (Theorem 4.1 on both passes)."""
    rng = np.random.default_rng(12)
    x = rng.uniform(size=(2, 12, 10))
    for s in (2, 4):
        y = O.upsample_2d(x, s)
        assert np.abs(y[:, ::s, ::s] - x).max() < 1e-12


def test_2d_row_pass_equals_1d_route():
    """A row pass is the 1-D reconstruction with channels {x, (x[p+1] - x[p-1]) N / (4 pi)}
    and multipliers {1, i n}: an image constant along columns isolates it."""
    rng = np.random.default_rng(13)
    w, h, s = 14, 6, 2
    row = rng.standard_normal(w)
    x = np.tile(row, (h, 1))
    y = O.upsample_2d(x, s)
    fd = (np.roll(row, -1) - np.roll(row, 1)) * w / (4 * np.pi)
    ch = O.Channels(N=w, kinds=[O.MULT_DERIV] * 2, orders=[0, 1])
    want = O.reconstruct_1d(ch, np.stack([row, fd]), s * w)[0]
    for r in range(s * h):
        assert np.abs(y[r] - want).max() < 1e-12


def test_2d_equals_fourier_window_form():
    """Each pass is shift-equivariant on the coarse grid, so the separable result is
    IFFT2( X[k_y mod h, k_x mod w] * Wh[k_y] * Ww[k_x] ), with W the DFT of the 1-D
    response to a unit impulse."""
    rng = np.random.default_rng(14)
    h, w, s = 8, 12, 2
    x = rng.uniform(size=(h, w))
    imp_w = np.zeros((h, w)); imp_w[:, 0] = 1.0      # impulse along rows, constant along columns
    imp_h = np.zeros((h, w)); imp_h[0, :] = 1.0
    Ww = np.fft.fft(O.upsample_2d(imp_w, s)[0])
    Wh = np.fft.fft(O.upsample_2d(imp_h, s)[:, 0])
    X = np.fft.fft2(x)
    ky = np.arange(s * h) % h
    kx = np.arange(s * w) % w
    Y = X[np.ix_(ky, kx)] * Wh[:, None] * Ww[None, :]
    want = np.fft.ifft2(Y).real
    assert np.abs(O.upsample_2d(x, s) - want).max() < 1e-12


def test_2d_smooth_separable_image_is_close():
    """For a smooth separable image the centred-difference channel is a good derivative,
    so the upsample is close to the true fine-grid image (pins the 1/(2h) scaling)."""
    h = w = 32
    s = 2
    u = lambda t: np.cos(2 * t) + 0.3 * np.sin(3 * t)
    v = lambda t: np.sin(t) + 0.2 * np.cos(4 * t)
    tc = 2 * np.pi * np.arange(h) / h
    tf = 2 * np.pi * np.arange(s * h) / (s * h)
    x = np.outer(u(tc), v(tc))
    y = O.upsample_2d(x, s)
    want = np.outer(u(tf), v(tf))
    assert np.abs(y - want).max() < 2e-2 * np.abs(want).max()


def test_psnr_helper():
    ref = np.zeros((4, 4))
    img = np.full((4, 4), 0.1)
    assert O.psnr(img, ref) == pytest.approx(20.0)


# ---------------------------------------------------------------- sampled evaluation
def test_evaluate_band_exact_recovery_off_grid():
    """A real trigonometric polynomial in the band, recovered from {f, f', f''} samples, is
    evaluated exactly at arbitrary (off-grid) points; so are its Hilbert transform and its
    derivative, whose closed forms are the coefficient-wise multipliers -i sgn n and i n."""
    N = 12
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    deg = (ch.mu - 1) // 2 - 1
    g, n, a = S.single_signal_fp64(seed=3, degree=deg, N=N)
    g = S.sample_channels(n, a, [S.deriv_multiplier(m) for m in range(3)], N, real=True)
    band = O.recover_band(ch, g)
    t = np.random.default_rng(4).uniform(0, 2 * np.pi, 37)
    E = np.exp(1j * np.outer(t, n))
    for op, order, mult in ((O.OUT_IDENTITY, 0, 1.0), (O.OUT_HILBERT, 0, -1j * np.sign(n)),
                            (O.OUT_DERIV, 1, 1j * n)):
        want = (E @ (mult * a)).real
        got = O.evaluate_band(band, ch.n1, t, op, order)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_evaluate_band_cos_to_sin_and_grid_equals_reconstruction():
    """Closed form: the band {cos 3t} gives H -> sin 3t and d/dt -> -3 sin 3t; on the output
    grid the sum is the reconstruction itself, including a grid coarser than the band."""
    n1 = -5
    a = np.zeros(11, dtype=complex)
    a[3 - n1] = a[-3 - n1] = 0.5
    t = np.linspace(0.1, 6.0, 29)
    assert np.abs(O.evaluate_band(a, n1, t, O.OUT_HILBERT) - np.sin(3 * t)).max() < 1e-14
    assert np.abs(O.evaluate_band(a, n1, t, O.OUT_DERIV, 1) + 3 * np.sin(3 * t)).max() < 1e-13
    rng = np.random.default_rng(8)
    ch = O.Channels(N=9, kinds=[O.MULT_DERIV, O.MULT_DERIV], orders=[0, 1])
    g = rng.standard_normal((2, 9))
    band = O.recover_band(ch, g)
    for n_out in (40, 7):
        tj = 2 * np.pi * np.arange(n_out) / n_out
        assert np.allclose(O.evaluate_band(band, ch.n1, tj), O.reconstruct_1d(ch, g, n_out)[0], atol=1e-12)


# ---------------------------------------------------------------- 2-D with three channels
def test_2d_three_channels_decimation_consistency():
    """With channels {x, Dx, D2x} (Section 5.2's experiments use three) the output still
    passes through the samples: out[s i, s j] = LR[i, j] (Theorem 4.1 on both passes)."""
    rng = np.random.default_rng(15)
    x = rng.uniform(size=(2, 10, 14))
    for s in (2, 3, 4):
        y = O.upsample_2d(x, s, M=3)
        assert np.abs(y[:, ::s, ::s] - x).max() < 1e-12


def test_2d_three_channels_row_pass_equals_1d_route():
    """A row pass is the 1-D reconstruction with channels {x, (x[p+1] - x[p-1]) N / (4 pi),
    (x[p+1] - 2 x[p] + x[p-1]) (N / 2 pi)^2} and multipliers {1, i n, (i n)^2}."""
    rng = np.random.default_rng(16)
    w, h, s = 15, 4, 3
    row = rng.standard_normal(w)
    x = np.tile(row, (h, 1))
    y = O.upsample_2d(x, s, M=3)
    fd = (np.roll(row, -1) - np.roll(row, 1)) * w / (4 * np.pi)
    fd2 = (np.roll(row, -1) - 2 * row + np.roll(row, 1)) * (w / (2 * np.pi)) ** 2
    ch = O.Channels(N=w, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    want = O.reconstruct_1d(ch, np.stack([row, fd, fd2]), s * w)[0]
    for r in range(s * h):
        assert np.abs(y[r] - want).max() < 1e-12


def test_2d_three_channels_fourier_window_form_and_smooth_image():
    """Shift-equivariance gives the FFT2 window form for three channels too; and a smooth
    separable image is reproduced closely at x3 (pins the (N / 2 pi)^2 scaling of D2)."""
    rng = np.random.default_rng(17)
    h, w, s = 9, 12, 3
    x = rng.uniform(size=(h, w))
    imp_w = np.zeros((h, w)); imp_w[:, 0] = 1.0
    imp_h = np.zeros((h, w)); imp_h[0, :] = 1.0
    Ww = np.fft.fft(O.upsample_2d(imp_w, s, M=3)[0])
    Wh = np.fft.fft(O.upsample_2d(imp_h, s, M=3)[:, 0])
    X = np.fft.fft2(x)
    Y = X[np.ix_(np.arange(s * h) % h, np.arange(s * w) % w)] * Wh[:, None] * Ww[None, :]
    assert np.abs(O.upsample_2d(x, s, M=3) - np.fft.ifft2(Y).real).max() < 1e-12
    n = 30
    u = lambda t: np.cos(2 * t) + 0.3 * np.sin(3 * t)
    v = lambda t: np.sin(t) + 0.2 * np.cos(4 * t)
    tc, tf = 2 * np.pi * np.arange(n) / n, 2 * np.pi * np.arange(s * n) / (s * n)
    y = O.upsample_2d(np.outer(u(tc), v(tc)), s, M=3)
    want = np.outer(u(tf), v(tf))
    assert np.abs(y - want).max() < 2e-2 * np.abs(want).max()
