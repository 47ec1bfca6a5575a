"""GPU parity: libmci (HIP, gfx950) against the FP64 oracle on the same seeded inputs.

Tolerances, per result, on both the relative L2 error ||y - y_ref|| / ||y_ref|| and the
element-wise error max|y - y_ref| / max|y_ref| (tests/parity.py):
  * FP64 plans: 1e-12 -- the transforms accumulate O(log n) roundings of 1.1e-16 with
    tables accurate to ~1e-16, and the per-residue tables are built in FP64;
  * FP32 plans: 1e-5  -- FP32 unit roundoff 6e-8 times a few tens of roundings along the
    path (log2 of the transform lengths, the M-term apply and the Bluestein chirps),
    times the growth of the equilibrated per-residue systems (condition <= ~20 here);
  * FP16 storage: the output's own rounding, 2^-11 relative, dominates: 1e-3.
Inputs are rounded once to the storage type and those rounded values go to both sides.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import images as SI
from synth import signals as S
from parity import check, check_rows

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401  (fails loudly without the built library)
    return torch


_OK = {"deriv": O.MULT_DERIV, "hilbert": O.MULT_HILBERT, "table": O.MULT_TABLE}
_OO = {"identity": O.OUT_IDENTITY, "hilbert": O.OUT_HILBERT, "deriv": O.OUT_DERIV}


def oracle_channels(channels, N, n1):
    kinds = [_OK[k] for k, _ in channels]
    orders = [int(v) if k != "table" else 0 for k, v in channels]
    tabs = None
    if any(k == "table" for k, _ in channels):
        mu = len(channels) * N
        tabs = np.zeros((len(channels), mu), dtype=complex)
        for i, (k, v) in enumerate(channels):
            if k == "table":
                tabs[i] = v
    return O.Channels(N=N, kinds=kinds, orders=orders, n1=n1, tables=tabs)


def run_case(torch, N, n_out, channels, ops=(("identity", 0),), real=True, precision="f32", storage="native",
             batch=3, n1=None, seed=0, allow_zero=False, g=None):
    from paper_1802_10291_amd import Plan1D
    M = len(channels)
    ch = oracle_channels(channels, N, n1)
    rng = np.random.default_rng(seed)
    if g is None:
        if real:
            g = rng.standard_normal((batch, M, N))
        else:
            g = rng.standard_normal((batch, M, N)) + 1j * rng.standard_normal((batch, M, N))
    np_dt = {"f64": np.float64, "f32": np.float32}[precision] if storage == "native" else np.float16
    if real:
        g_store = g.astype(np_dt)
        g_ref = g_store.astype(np.float64)
        g_dev = torch.from_numpy(g_store).cuda()
    else:
        parts = np.stack([g.real, g.imag], axis=-1).astype(np_dt)
        g_ref = parts[..., 0].astype(np.float64) + 1j * parts[..., 1].astype(np.float64)
        g_dev = torch.from_numpy(np.ascontiguousarray(parts)).cuda()
    plan = Plan1D(N=N, n_out=n_out, channels=channels, ops=ops, n1=n1, real=real, precision=precision,
                  storage=storage, allow_singular_zero=allow_zero)
    y = plan.reconstruct(g_dev)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    if not real:
        y = y[..., 0] + 1j * y[..., 1]
    want = O.reconstruct_1d(ch, g_ref, n_out, ops=[_OO[o] for o, _ in ops], op_orders=[int(v) for _, v in ops],
                            allow_singular_zero=allow_zero)
    return y, want, plan


def assert_parity(y, want, tol):
    """Every output row (signal, operator) within tol by relative L2 and element-wise."""
    B, n_ops = y.shape[0], y.shape[1]
    err, _ = check_rows(y.reshape(B * n_ops, -1), want.reshape(B * n_ops, -1), tol)
    return err


# ----------------------------------------------------------------------- single signal, FP64
def test_single_signal_fp64_exact(torch_cuda):
    """The single-signal FP64 workload: f of degree 127 from {f, f'} with 128 samples each,
    f and Hf on 4096 points; exact recovery and oracle match at 1e-12."""
    g, n, a = S.single_signal_fp64(seed=1, degree=127, N=128)
    y, want, plan = run_case(torch_cuda, 128, 4096, [("deriv", 0), ("deriv", 1)],
                             ops=[("identity", 0), ("hilbert", 0)], precision="f64", g=g[None])
    assert plan.info.n1 == -127
    assert_parity(y, want, TOL["f64"])
    tj = 2 * np.pi * np.arange(4096) / 4096
    E = np.exp(1j * np.outer(tj, n))
    f = (E @ a).real
    Hf = (E @ (-1j * np.sign(n) * a)).real
    check(y[0, 0], f, 1e-12)
    check(y[0, 1], Hf, 1e-12)


# ----------------------------------------------------------------------- parity sweep
SWEEP = [
    # N, n_out, channels, ops, real
    (16, 64, [("deriv", 0), ("deriv", 1)], [("identity", 0)], True),
    (24, 96, [("deriv", 0), ("deriv", 1), ("deriv", 2)], [("identity", 0), ("hilbert", 0)], True),
    (13, 52, [("deriv", 0), ("deriv", 1), ("deriv", 2)], [("identity", 0)], True),        # Bluestein N
    (11, 97, [("deriv", 0), ("hilbert", 0)], [("identity", 0), ("deriv", 1)], False),     # Bluestein n_out
    (20, 30, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], [("identity", 0)], True),  # n_out < mu folds
    (9, 36, [("deriv", 0)], [("identity", 0), ("hilbert", 0)], True),
    (1, 8, [("deriv", 0), ("deriv", 1)], [("identity", 0)], True),                        # one sample per channel
    (7, 1, [("deriv", 0), ("deriv", 1)], [("identity", 0)], False),                       # one output point
    (100, 700, [("deriv", 0), ("deriv", 1), ("deriv", 2)], [("identity", 0), ("deriv", 2)], True),
    (128, 512, [("deriv", 0), ("deriv", 1)], [("identity", 0)], True),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(SWEEP)))
def test_parity_sweep(torch_cuda, precision, case):
    N, n_out, channels, ops, real = SWEEP[case]
    y, want, _ = run_case(torch_cuda, N, n_out, channels, ops=ops, real=real, precision=precision, seed=case)
    assert_parity(y, want, TOL[precision])


def test_parity_random_table_multipliers(torch_cuda):
    rng = np.random.default_rng(7)
    for M in (2, 3, 4):
        N = 10
        tabs = [("table", rng.standard_normal(M * N) + 1j * rng.standard_normal(M * N)) for _ in range(M)]
        for precision in ("f64", "f32"):
            y, want, plan = run_case(torch_cuda, N, 64, tabs, real=False, precision=precision, seed=M)
            assert plan.info.max_cond <= 25.0
            assert_parity(y, want, TOL[precision])


@pytest.mark.parametrize("N,n_out,M,real", [(1366, 16384, 3, True), (1024, 4096, 2, True), (100, 700, 3, True),
                                           (24, 96, 2, False)])
def test_strided_batch_matches_dense(torch_cuda, N, n_out, M, real):
    """mci_reconstruct_1d_strided on signals inside longer rows (a view of g and of y with a
    batch stride) gives the dense call's outputs bit for bit, on the single-pass, real-mode
    and multi-pass paths and for complex samples, and leaves the gaps between output rows
    untouched; strides that are not multiples of 4 or shorter than a signal are rejected."""
    from paper_1802_10291_amd import MCIError, Plan1D
    torch = torch_cuda
    chans = [("deriv", m) for m in range(M)]
    plan = Plan1D(N=N, n_out=n_out, channels=chans, real=real)
    c = 1 if real else 2
    n_in, n_o = M * N * c, n_out * c
    B = 5
    rng = np.random.default_rng(N + M)
    g = torch.from_numpy(rng.standard_normal((B, n_in)).astype(np.float32)).cuda()
    ld_g = n_in + 4 + (-n_in) % 4
    ld_y = n_o + 8 + (-n_o) % 4
    big_g = torch.zeros((B, ld_g), device="cuda")
    big_g[:, :n_in] = g
    big_y = torch.full((B, ld_y), float("nan"), device="cuda")
    tail = (M, N) if real else (M, N, 2)
    gv = big_g[:, :n_in].unflatten(1, tail)
    yv = big_y[:, :n_o].unflatten(1, (1, n_out) if real else (1, n_out, 2))
    assert not gv.is_contiguous() and not yv.is_contiguous()
    plan.reconstruct(gv, out=yv)
    dense = plan.reconstruct(g.unflatten(1, tail).contiguous())
    assert torch.equal(yv, dense)
    assert torch.isnan(big_y[:, n_o:]).all()
    with pytest.raises(MCIError):
        plan.reconstruct(big_g[:, : n_in].unflatten(1, tail), out=big_y[:, 2: n_o + 2].unflatten(
            1, (1, n_out) if real else (1, n_out, 2)))      # misaligned output start
    from paper_1802_10291_amd import _lib as L
    ws = torch.empty(L.mci_workspace_size_strided(plan.handle, B) + 64, dtype=torch.uint8, device="cuda")
    for bad_g, bad_y in ((ld_g + 2, ld_y), (ld_g, n_o - 4)):
        with pytest.raises(MCIError):
            L.mci_reconstruct_1d_strided(plan.handle, big_g.data_ptr(), bad_g, big_y.data_ptr(), bad_y, B,
                                         ws.data_ptr(), ws.numel(), 0)


@pytest.mark.parametrize("N,n_out,M,n1", [(171, 2048, 3, None), (683, 8192, 3, None), (683, 16384, 3, None),
                                          (601, 8192, 2, None), (171, 2048, 2, -100), (255, 8192, 4, None)])
def test_fused_odd_n_parity(torch_cuda, N, n_out, M, n1):
    """Odd N on the single-pass kernel: the channel DFT is the length-N transform of the real
    samples (Bluestein at 512 or split Bluestein at 1024), with no even/odd recovery; against
    the oracle element by element at 1e-5, and against the multi-kernel path."""
    from paper_1802_10291_amd import Plan1D
    chans = [("deriv", m) for m in range(M)]
    y, want, plan = run_case(torch_cuda, N, n_out, chans, n1=n1, seed=N + M)
    assert plan.info.path == 1 and "odd N" in plan.kernel_name(), plan.kernel_name()
    assert_parity(y, want, TOL["f32"])


def test_parity_f16_storage(torch_cuda):
    y, want, _ = run_case(torch_cuda, 64, 256, [("deriv", 0), ("deriv", 1)], storage="f16", batch=4, seed=3)
    assert_parity(y, want, TOL["f16"])


def test_hilbert_only_singular_and_remark_3_4(torch_cuda):
    from paper_1802_10291_amd import MCIError, Plan1D
    with pytest.raises(MCIError) as ei:
        Plan1D(N=9, n_out=40, channels=[("hilbert", 0)], real=False)
    assert ei.value.status == 2
    n, a = S.random_bandlimited(seed=3, n_lo=-4, n_hi=4)
    a[4] = 0.0
    g = S.sample_channels(n, a, [lambda k: -1j * np.sign(k)], 9)[None]
    y, want, plan = run_case(torch_cuda, 9, 40, [("hilbert", 0)], real=False, precision="f64", g=g, allow_zero=True)
    assert plan.info.n_singular == 1 and plan.info.first_singular == 0
    assert_parity(y, want, TOL["f64"])
    truth = np.exp(1j * np.outer(2 * np.pi * np.arange(40) / 40, n)) @ a
    assert np.abs(y[0, 0] - truth).max() < 1e-12


def test_ill_conditioned_rejected(torch_cuda):
    from paper_1802_10291_amd import MCIError, Plan1D
    with pytest.raises(MCIError) as ei:
        Plan1D(N=64, n_out=256, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)], cond_max=1.5)
    assert ei.value.status == 3
    p = Plan1D(N=64, n_out=256, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)])
    assert 1.0 <= p.info.max_cond < 100.0


def test_batch_zero_is_noop(torch_cuda):
    from paper_1802_10291_amd import Plan1D
    p = Plan1D(N=16, n_out=64, channels=[("deriv", 0), ("deriv", 1)])
    g = torch_cuda.zeros((0, 2, 16), device="cuda")
    assert p.reconstruct(g).shape == (0, 1, 64)


def test_misaligned_buffers_rejected(torch_cuda):
    """Device buffers must be 16-byte aligned (the kernels use vector accesses): a contiguous
    view that starts one element into its allocation is refused with an argument error, and
    the same values at an aligned address reconstruct normally."""
    from paper_1802_10291_amd import MCIError, Plan1D, Plan2D
    torch = torch_cuda
    p = Plan1D(N=1366, n_out=16384, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)])
    raw = torch.randn(2 * 3 * 1366 + 1, device="cuda")
    g_bad = raw[1:].view(2, 3, 1366)
    assert g_bad.is_contiguous() and g_bad.data_ptr() % 16 != 0
    with pytest.raises(MCIError, match="INVALID_ARG"):
        p.reconstruct(g_bad)
    y = p.reconstruct(g_bad.clone())
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    q = Plan2D(64, 64, 2)
    raw2 = torch.rand(64 * 64 + 1, device="cuda")
    with pytest.raises(MCIError, match="INVALID_ARG"):
        q.upsample(raw2[1:].view(1, 64, 64))


# ----------------------------------------------------------------------- batched FP32 workload
def test_batched_fp32_small_batch_full_parity(torch_cuda):
    """The batched FP32 workload's shape (M = 3 derivative channels, N = 1366, band
    [-2048, 2049], 16384 output points) on a small batch, every output compared."""
    g = S.smooth_noisy_batch(0, 4, 3, 1366, 8192)
    y, want, plan = run_case(torch_cuda, 1366, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2)], g=g)
    assert plan.info.n1 == -2048
    err = assert_parity(y, want, TOL["f32"])
    print("batched-fp32 small batch rel L2:", err)


# ----------------------------------------------------------------------- 2-D
@pytest.mark.parametrize("s", [2, 4])
def test_2d_parity_small(torch_cuda, s):
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(0, 2, 48, 40)
    for precision, tol in (("f64", 1e-12), ("f32", 1e-5)):
        x = lr.astype(np.float64 if precision == "f64" else np.float32)
        plan = Plan2D(48, 40, s, precision=precision)
        hr = plan.upsample(torch_cuda.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
        want = O.upsample_2d(x.astype(np.float64), s)
        check_rows(hr, want, tol)
        assert np.abs(hr[:, ::s, ::s] - x).max() <= (1e-12 if precision == "f64" else 1e-5)


# ----------------------------------------------------------------------- fused single-pass kernel
FUSED = [
    # N, n_out, channels, n1
    (1366, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2)], None),    # Bluestein forward (H = 683)
    (2048, 16384, [("deriv", 0), ("deriv", 1)], None),                  # direct forward (H = 1024)
    (1000, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2)], None),    # Bluestein, PF = 1024
    (1022, 8192, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], None),  # M = 4, P = 2048
    (1366, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2)], -2500),   # shifted band
    (2048, 16384, [("deriv", 0), ("hilbert", 0)], None),                # Hilbert channel
    (1000, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 100),     # band not containing 0
    (1100, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2)], None),    # split Bluestein, H = 550
    (1200, 16384, [("deriv", 0)], None),                                # split Bluestein, M = 1, H = 600
    (1024, 16384, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], None),  # 512-point forward, M = 4
    (1024, 8192, [("deriv", 0), ("deriv", 1)], None),                   # 512-point forward, P = 2048
    (342, 4096, [("deriv", 0), ("deriv", 1), ("deriv", 2)], None),      # Bluestein at 512 (H = 171), P = 1024
    (300, 4096, [("deriv", 0), ("deriv", 1)], -20),                     # Bluestein at 512 (H = 150), shifted band
    (1024, 12288, [("deriv", 0), ("deriv", 1), ("deriv", 2)], None),    # 3072-point output (radix 12 last)
    (768, 12288, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], None),  # Bluestein 1024, P = 3072
    (1536, 12288, [("deriv", 0), ("deriv", 1)], -1500),                 # Bluestein 2048, P = 3072, shifted band
    (512, 8192, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], None),  # power-of-two H = 256 by Bluestein
    (256, 2048, [("deriv", 0), ("deriv", 1)], None),                    # one output transform (Q = 2), P = 1024
    (768, 6144, [("deriv", 0), ("deriv", 1)], None),                    # Q = 2, P = 3072, Bluestein 1024
    (384, 6144, [("deriv", 0), ("hilbert", 0)], None),                  # Q = 2, P = 3072, Hilbert channel
    (86, 1024, [("deriv", 0), ("deriv", 1), ("deriv", 2)], None),       # Q = 2, P = 512 (H = 43)
    (192, 3072, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], None),  # Q = 2, P = 1536 (radix 3 last)
    (384, 3072, [("deriv", 0), ("deriv", 1)], -300),                    # Q = 2, P = 1536, shifted band
]


@pytest.mark.parametrize("case", range(len(FUSED)))
def test_fused_kernel_parity(torch_cuda, case):
    N, n_out, channels, n1 = FUSED[case]
    M = len(channels)
    g = S.smooth_noisy_batch(10 * case, 3, M, N, 2 * N)
    if any(k == "hilbert" for k, _ in channels):
        g = np.random.default_rng(case).standard_normal((3, M, N))
    y, want, plan = run_case(torch_cuda, N, n_out, channels, g=g, n1=n1)
    assert plan.info.path == 1, "expected the fused kernel"
    assert_parity(y, want, TOL["f32"])


def test_fused_matches_multipass(torch_cuda, monkeypatch):
    """Both paths compute the same thing: compare them on a batch bigger than the grid."""
    from paper_1802_10291_amd import Plan1D
    g = torch_cuda.from_numpy(S.smooth_noisy_batch(0, 64, 3, 1366, 8192)).cuda()
    chans = [("deriv", 0), ("deriv", 1), ("deriv", 2)]
    fused = Plan1D(N=1366, n_out=16384, channels=chans)
    monkeypatch.setenv("MCI_DISABLE_FUSED", "1")
    multi = Plan1D(N=1366, n_out=16384, channels=chans)
    assert fused.info.path == 1 and multi.info.path == 0
    a = fused.reconstruct(g).cpu().numpy().astype(np.float64)
    b = multi.reconstruct(g).cpu().numpy().astype(np.float64)
    check_rows(a.reshape(64, -1), b.reshape(64, -1), 2e-6)


# ----------------------------------------------------------------------- fused 2-D line passes
@pytest.mark.parametrize("h,w,s", [(256, 256, 2), (128, 128, 4), (64, 128, 2), (128, 64, 4), (256, 128, 4),
                                   (32, 32, 2), (48, 48, 4), (96, 48, 2), (192, 192, 2), (384, 384, 2),
                                   (512, 512, 2), (512, 384, 4), (32, 512, 2)])
def test_2d_line_pass_parity(torch_cuda, h, w, s):
    """Columns then rows through the polyphase-window line passes, against the FP64 oracle
    (rows then columns: the two passes act on different axes and commute)."""
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(7, 2 if h * w <= 256 * 256 else 1, h, w)
    plan = Plan2D(h, w, s)
    assert plan.info.path == 1
    hr = plan.upsample(torch_cuda.from_numpy(lr).cuda()).cpu().numpy().astype(np.float64)
    want = O.upsample_2d(lr.astype(np.float64), s)
    check_rows(hr, want, 1e-5)
    assert np.abs(hr[:, ::s, ::s] - lr).max() <= 1e-5


@pytest.mark.parametrize("h,w,s", [(64, 64, 3), (96, 128, 3), (48, 40, 3), (128, 128, 2), (64, 32, 4)])
def test_2d_three_channels_parity(torch_cuda, h, w, s):
    """Channels {x, Dx, D2x} per line (Section 5.2's experiments: x3), through the line passes
    (sides in the line-length set) or the multi-pass route (a side of 40), against the FP64
    oracle; the output passes through the samples."""
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(21, 2, h, w)
    plan = Plan2D(h, w, s, channels=3)
    assert plan.info.path == (0 if 40 in (h, w) else 1)
    hr = plan.upsample(torch_cuda.from_numpy(lr).cuda()).cpu().numpy().astype(np.float64)
    want = O.upsample_2d(lr.astype(np.float64), s, M=3)
    check_rows(hr, want, 1e-5)
    assert np.abs(hr[:, ::s, ::s] - lr).max() <= 1e-5


@pytest.mark.parametrize("h,w,s,M", [(256, 256, 2, 2), (128, 128, 4, 2), (64, 96, 3, 3), (48, 32, 2, 2)])
def test_2d_sample_rows_passed_through(torch_cuda, monkeypatch, h, w, s, M):
    """Interpolation consistency makes the columns pass's polyphase row 0 the input itself, so
    the FP32 line passes can skip computing it, with the rows pass reading those lines from the
    input (the default at scale 2, MCI_LP_ZR=1 at the others).  Against the form that computes
    every row (MCI_LP_FULL_COLUMNS=1) and the oracle; ragged batch (3 images) so the rows
    pass's 32-line blocks straddle images."""
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(31, 3, h, w)
    if s != 2:
        assert "passed through" not in Plan2D(h, w, s, channels=M).kernel_name()
        monkeypatch.setenv("MCI_LP_ZR", "1")
    plan = Plan2D(h, w, s, channels=M)
    assert "sample rows passed through" in plan.kernel_name()
    monkeypatch.setenv("MCI_LP_FULL_COLUMNS", "1")
    full = Plan2D(h, w, s, channels=M)
    assert "passed through" not in full.kernel_name() and full.info.path == 1
    x = torch_cuda.from_numpy(lr).cuda()
    a = plan.upsample(x).cpu().numpy().astype(np.float64)
    b = full.upsample(x).cpu().numpy().astype(np.float64)
    want = O.upsample_2d(lr.astype(np.float64), s, M=M)
    check_rows(a, want, 1e-5)
    check_rows(a, b, 2e-6)
    assert np.abs(a[:, ::s, ::s] - lr).max() <= 1e-5


@pytest.mark.parametrize("h,w,s", [(256, 256, 2), (128, 128, 4), (64, 96, 3), (48, 32, 2), (96, 64, 4)])
def test_2d_f16_storage(torch_cuda, h, w, s):
    """FP16 images in and out (FP32 arithmetic): the columns pass reads four halves per load
    and the rows pass writes a position's s outputs in one store (s = 2, 4); against the
    oracle on the FP16-rounded input, within FP16's output rounding."""
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(51 + s, 3, h, w).astype(np.float16)
    plan = Plan2D(h, w, s, storage="f16")
    assert plan.info.path == 1
    hr = plan.upsample(torch_cuda.from_numpy(lr).cuda())
    assert hr.dtype == torch_cuda.float16
    hr = hr.cpu().numpy().astype(np.float64)
    check_rows(hr, O.upsample_2d(lr.astype(np.float64), s), TOL["f16"])


def test_2d_three_channels_fp64_exact(torch_cuda):
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(22, 2, 30, 36).astype(np.float64)
    plan = Plan2D(30, 36, 3, precision="f64", channels=3)
    hr = plan.upsample(torch_cuda.from_numpy(lr).cuda()).cpu().numpy()
    check_rows(hr, O.upsample_2d(lr, 3, M=3), 1e-12)


def test_2d_line_pass_ragged_batch(torch_cuda):
    """Batch sizes that leave partial 32-line blocks in the row pass."""
    from paper_1802_10291_amd import Plan2D
    lr = SI.random_field_images(11, 3, 64, 64)
    plan = Plan2D(64, 64, 2)
    for b in (1, 3):
        hr = plan.upsample(torch_cuda.from_numpy(lr[:b]).cuda()).cpu().numpy().astype(np.float64)
        want = O.upsample_2d(lr[:b].astype(np.float64), 2)
        check_rows(hr, want, 1e-5)


# ----------------------------------------------------------------------- Table 1 on the GPU
def _table1_rows():
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows.append((int(v[0]), int(v[1]), int(v[2]), int(v[3]), float(v[5]), float(v[6])))
    return rows


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_table1_on_gpu(torch_cuda, precision):
    """Table 1 (Section 5.1) from the GPU: the 16 channel sets ({f}, {f, Hf}, {f, f', f''} at
    mu = 16 .. 108) reconstruct f and Hf of the rational test signal on 2048 points (real
    mode, output operators identity and -i sgn n).  FP64 plans give the printed delta_1 and
    delta_2 to 4 significant digits (the mu = 96 {f, Hf} delta_2 recomputes to 0.3869e-2,
    the misprint the oracle pins also exclude); FP32 plans stay within 1e-5 of the FP64
    deltas, which is the FP32 parity bound since both deltas are normalised by the same
    reference norm."""
    from paper_1802_10291_amd import Plan1D
    torch = torch_cuda
    c = S.phi_coeffs()
    tg = 2 * np.pi * np.arange(2048) / 2048
    F, HF = S.phi_samples("f", tg, c), S.phi_samples("H", tg, c)
    dt = {"f64": np.float64, "f32": np.float32}[precision]
    for mu, nf, nh, nd, d1, d2 in _table1_rows():
        if nh:
            channels, names = [("deriv", 0), ("hilbert", 0)], ["f", "H"]
        elif nd:
            channels, names = [("deriv", 0), ("deriv", 1), ("deriv", 2)], ["f", "d1", "d2"]
        else:
            channels, names = [("deriv", 0)], ["f"]
        N = mu // len(channels)
        tp = 2 * np.pi * np.arange(N) / N
        g = np.stack([S.phi_samples(k, tp, c) for k in names])[None].astype(dt)
        plan = Plan1D(N=N, n_out=2048, channels=channels, ops=[("identity", 0), ("hilbert", 0)], real=True,
                      precision=precision)
        y = plan.reconstruct(torch.from_numpy(g).cuda())
        torch.cuda.synchronize()
        y = y.cpu().numpy().astype(np.float64)[0]
        want = O.reconstruct_1d(oracle_channels(channels, N, None), g.astype(np.float64), 2048,
                                ops=[O.OUT_IDENTITY, O.OUT_HILBERT])[0]
        assert_parity(y[None], want[None], TOL[precision])
        e1 = np.linalg.norm(F - y[0]) / np.linalg.norm(F)
        e2 = np.linalg.norm(HF - y[1]) / np.linalg.norm(HF)
        if precision == "f64":
            assert float(f"{e1:.4g}") == pytest.approx(d1, rel=1e-9), (mu, names, e1, d1)
            want2 = 0.003869 if (mu == 96 and nh) else d2
            assert float(f"{e2:.4g}") == pytest.approx(want2, rel=1e-9), (mu, names, e2, d2)
        else:
            w1 = np.linalg.norm(F - want[0]) / np.linalg.norm(F)
            w2 = np.linalg.norm(HF - want[1]) / np.linalg.norm(HF)
            assert abs(e1 - w1) <= 1e-5 and abs(e2 - w2) <= 1e-5, (mu, names, e1, w1, e2, w2)


def test_fused_kernel_table_channels(torch_cuda):
    """The fused kernel with table multipliers: scaled derivatives (i n / N)^m given as
    tables over the band."""
    N, n_out, M = 1366, 16384, 3
    mu = M * N
    n = np.arange(O.default_n1(mu), O.default_n1(mu) + mu)
    channels = [("table", (1j * n / N) ** m) for m in range(M)]
    g = S.smooth_noisy_batch(70, 3, M, N, 2 * N)
    y, want, plan = run_case(torch_cuda, N, n_out, channels, g=g)
    assert plan.info.path == 1, "expected the fused kernel"
    assert_parity(y, want, TOL["f32"])
