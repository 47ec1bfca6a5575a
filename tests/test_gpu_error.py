"""Averaged approximation error on the GPU (``mci_averaged_error``) and its bound
(``mci_error_bound``, eq. errorestimate) against the FP64 oracle.

The oracle's ``averaged_error`` evaluates eq. averageerror term by term and is pinned in the
CPU suite against Theorem 4.4 itself (the phase average of actual reconstruction errors).
Tolerances on eps (relative): 1e-12 for FP64 inputs, 1e-5 for FP32 inputs (each |a(n)|^2 w(n)
term is rounded once to FP32 and the sums run in FP32 over a few hundred terms per thread
before an FP64 combine).  The least-error plan is compared where the two best errors differ
by more than that tolerance, since closer ones may legitimately swap.
"""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

_OK = {"deriv": O.MULT_DERIV, "hilbert": O.MULT_HILBERT}

CANDIDATES = [
    # (N, channels, n1 offset from the default)
    (48, [("deriv", 0)], 0),
    (24, [("deriv", 0), ("deriv", 1)], 0),
    (16, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 0),
    (24, [("deriv", 0), ("hilbert", 0)], 0),
    (24, [("deriv", 0), ("deriv", 1)], 3),
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401  (fails loudly without the built library)
    return torch


def _plans(cands, precision="f32"):
    from paper_1802_10291_amd import Plan1D
    out = []
    for N, channels, shift in cands:
        mu = N * len(channels)
        n1 = O.default_n1(mu) + shift
        out.append((Plan1D(N=N, n_out=2 * mu, channels=channels, n1=n1, precision=precision),
                    O.Channels(N=N, kinds=[_OK[k] for k, _ in channels], orders=[int(v) for _, v in channels], n1=n1)))
    return out


def _spectra(n_sig, n_lo, n_span, seed):
    """Signal 0: the rational test signal of Section 5.1 (f = Re phi); the others random with
    decaying coefficients, some real-valued (a(-n) = conj a(n))."""
    from synth import signals as S
    rng = np.random.default_rng(seed)
    n = np.arange(n_lo, n_lo + n_span)
    a = np.zeros((n_sig, n_span), dtype=np.complex128)
    c = S.phi_coeffs(max(abs(n_lo), abs(n_lo + n_span - 1)) + 1)
    a[0] = np.where(n == 0, c[0], c[np.abs(n)] / 2)
    for s in range(1, n_sig):
        decay = rng.uniform(0.02, 0.2)
        a[s] = np.exp(-decay * np.abs(n)) * (rng.standard_normal(n_span) + 1j * rng.standard_normal(n_span))
        if s % 2:
            a[s] = 0.5 * (a[s] + np.conj(a[s][::-1]))
    return n, a


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_averaged_error_matches_oracle(torch_cuda, precision, tol):
    from paper_1802_10291_amd import averaged_error
    torch = torch_cuda
    plans = _plans(CANDIDATES)
    n_lo, n_span, n_sig = -150, 301, 11       # 11 signals: an 8-signal workgroup and a ragged one
    n, a = _spectra(n_sig, n_lo, n_span, seed=4)
    cdt = np.complex128 if precision == "f64" else np.complex64
    a_dev = torch.from_numpy(a.astype(cdt)).cuda()
    eps, best = averaged_error([p for p, _ in plans], a_dev, n_lo)
    eps, best = eps.cpu().numpy(), best.cpu().numpy()
    a_ref = a.astype(cdt).astype(np.complex128)
    want = np.array([[O.averaged_error(ch, n, a_ref[s]) for _, ch in plans] for s in range(n_sig)])
    assert np.all(np.abs(eps - want) <= tol * want), np.abs(eps / want - 1).max()
    for s in range(n_sig):
        order = np.argsort(want[s])
        if want[s, order[1]] - want[s, order[0]] > 4 * tol * want[s, order[1]]:
            assert best[s] == order[0], (s, want[s], eps[s])


def test_bandlimited_signal_has_zero_error(torch_cuda):
    """A signal inside a plan's band is recovered exactly (Theorem 3.3): its averaged error
    under that plan is 0, and nonzero under a plan whose band misses part of it."""
    from paper_1802_10291_amd import averaged_error
    torch = torch_cuda
    plans = _plans([(24, [("deriv", 0), ("deriv", 1)], 0), (24, [("deriv", 0), ("deriv", 1)], 10)])
    n_lo, n_span = -30, 61
    n = np.arange(n_lo, n_lo + n_span)
    rng = np.random.default_rng(9)
    a = np.where((n >= -23) & (n <= 24), rng.standard_normal(n_span) + 1j * rng.standard_normal(n_span), 0)
    eps, best = averaged_error([p for p, _ in plans], torch.from_numpy(a[None]).cuda(), n_lo)
    eps = eps.cpu().numpy()[0]
    assert eps[0] == 0.0 and eps[1] > 0.1
    assert int(best.cpu()[0]) == 0


def test_averaged_error_rejects(torch_cuda):
    from paper_1802_10291_amd import MCIError, Plan1D, averaged_error
    torch = torch_cuda
    a = torch.zeros((2, 10), dtype=torch.complex64, device="cuda")
    tab = 1j * np.arange(-15, 17)            # b(n) = i n on the band [-15, 16]: invertible with f
    p_tab = Plan1D(N=16, n_out=32, channels=[("deriv", 0), ("table", tab)])
    with pytest.raises(MCIError, match="UNSUPPORTED"):
        averaged_error([p_tab], a, -5)
    p_sing = Plan1D(N=9, n_out=40, channels=[("hilbert", 0)], real=False, allow_singular_zero=True)
    with pytest.raises(MCIError, match="SINGULAR"):
        averaged_error([p_sing], a, -5)
    p_ok = Plan1D(N=16, n_out=32, channels=[("deriv", 0)])
    with pytest.raises(MCIError):
        averaged_error([p_ok] * 17, a, -5)
    with pytest.raises(ValueError):
        averaged_error([p_ok], torch.zeros((2, 10), dtype=torch.float32, device="cuda"), -5)


def test_averaged_error_full_size_sampled(torch_cuda):
    """The benchmark's shape: 4096 signals with coefficients on |n| <= 8192 (16385 per signal)
    scored against 8 plans of about 4098 samples each; 4 sampled signals against the oracle."""
    from paper_1802_10291_amd import Plan1D, averaged_error
    from synth import signals as S
    torch = torch_cuda
    cands = [(4098, [("deriv", 0)], 0), (2049, [("deriv", 0), ("deriv", 1)], 0),
             (1366, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 0), (2049, [("deriv", 0), ("hilbert", 0)], 0),
             (1025, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], 0),
             (2049, [("deriv", 0), ("deriv", 1)], 64), (4098, [("deriv", 0)], -64),
             (1366, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 32)]
    plans = _plans(cands)
    n_max, n_sig, pool = 8192, 4096, 64
    n_lo, n_span = -n_max, 2 * n_max + 1
    rng = np.random.default_rng(77)
    host = np.empty((pool, n_span), dtype=np.complex64)
    for s in range(pool):
        nn, c = S.smooth_noisy_spectrum(rng, n_max)
        host[s] = c
    a = torch.from_numpy(host).cuda().repeat(n_sig // pool, 1)
    eps, best = averaged_error([p for p, _ in plans], a, n_lo)
    eps = eps.cpu().numpy()
    n = np.arange(n_lo, n_lo + n_span)
    for s in (0, 17, 1000, 4095):
        ref = host[s % pool].astype(np.complex128)
        want = np.array([O.averaged_error(ch, n, ref) for _, ch in plans])
        assert np.all(np.abs(eps[s] - want) <= 1e-5 * want), (s, eps[s], want)
    assert np.isfinite(eps).all()


# ------------------------------------------------------------------ the bound (eq. errorestimate)
def test_plan_omega_matches_oracle(torch_cuda):
    """Omega_m of every candidate plan (the definition after Theorem 4.4) from the GPU's FP64
    inverse tables equals the oracle's, whose closed forms are pinned in the CPU suite."""
    for plan, ch in _plans(CANDIDATES, "f64"):
        got = np.array(plan.omega())
        want = O.omega(ch)
        assert np.allclose(got, want, rtol=1e-12, atol=0), (got, want)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_error_bound_matches_oracle(torch_cuda, precision, tol):
    """The bound of eq. errorestimate per (signal, plan) against the oracle's term-by-term
    evaluation, 11 signals (a full and a ragged workgroup) x 5 plans; it bounds the averaged
    error computed by the same call's sibling, and is 0 for a bandlimited signal."""
    from paper_1802_10291_amd import averaged_error, error_bound
    torch = torch_cuda
    plans = _plans(CANDIDATES)
    n_lo, n_span, n_sig = -150, 301, 11
    n, a = _spectra(n_sig, n_lo, n_span, seed=6)
    cdt = np.complex128 if precision == "f64" else np.complex64
    a_dev = torch.from_numpy(a.astype(cdt)).cuda()
    bound = error_bound([p for p, _ in plans], a_dev, n_lo).cpu().numpy()
    eps, _ = averaged_error([p for p, _ in plans], a_dev, n_lo)
    eps = eps.cpu().numpy()
    a_ref = a.astype(cdt).astype(np.complex128)
    want = np.array([[O.error_bound(ch, n, a_ref[s]) for _, ch in plans] for s in range(n_sig)])
    assert np.all(np.abs(bound - want) <= tol * want), np.abs(bound / want - 1).max()
    assert np.all(bound >= eps * (1 - 2 * tol))
    inband = (n >= -23) & (n <= 24)
    a0 = np.where(inband, a[1], 0)[None].astype(cdt)
    b0 = error_bound([plans[1][0]], torch.from_numpy(a0).cuda(), n_lo).cpu().numpy()
    assert b0[0, 0] == 0.0


def test_error_bound_full_size_sampled(torch_cuda):
    """The averaged-error benchmark's shape for the bound: 4096 signals x 16385 coefficients x
    4 plans of about 4098 samples; 3 sampled signals against the oracle, all finite."""
    from paper_1802_10291_amd import error_bound
    from synth import signals as S
    torch = torch_cuda
    cands = [(4098, [("deriv", 0)], 0), (2049, [("deriv", 0), ("deriv", 1)], 0),
             (1366, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 0), (2049, [("deriv", 0), ("hilbert", 0)], 0)]
    plans = _plans(cands)
    n_max, n_sig, pool = 8192, 4096, 32
    n_lo, n_span = -n_max, 2 * n_max + 1
    rng = np.random.default_rng(78)
    host = np.empty((pool, n_span), dtype=np.complex64)
    for s in range(pool):
        host[s] = S.smooth_noisy_spectrum(rng, n_max)[1]
    a = torch.from_numpy(host).cuda().repeat(n_sig // pool, 1)
    bound = error_bound([p for p, _ in plans], a, n_lo).cpu().numpy()
    n = np.arange(n_lo, n_lo + n_span)
    for s in (0, 1001, 4095):
        ref = host[s % pool].astype(np.complex128)
        want = np.array([O.error_bound(ch, n, ref) for _, ch in plans])
        assert np.all(np.abs(bound[s] - want) <= 1e-5 * want), (s, bound[s], want)
    assert np.isfinite(bound).all()
