"""The allocation-free entry point mci_averaged_error_noalloc, through the C ABI, against
mci_averaged_error (the same kernels with a caller workspace): identical eps and least-error
plans on two calls in a row, the second with fewer coefficients, fewer signals and fewer
plans than the first (so stale contents of the shared static array would show), and a size
beyond the static array rejected before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401  (fails loudly without the built library)
    return torch


def _spectra(rng, n_sig, n_span):
    n = np.arange(n_span) - n_span // 2
    a = (rng.standard_normal((n_sig, n_span)) + 1j * rng.standard_normal((n_sig, n_span))) * \
        np.exp(-rng.uniform(0.001, 0.05, (n_sig, 1)) * np.abs(n))
    return a.astype(np.complex64), -(n_span // 2)


def _call_both(torch, plans, a_host, n_lo):
    from paper_1802_10291_amd import _lib
    a = torch.from_numpy(a_host).cuda()
    n_sig, n_span = a.shape
    handles = [p.handle for p in plans]
    stream = int(torch.cuda.current_stream().cuda_stream)
    eps_ref = torch.full((n_sig, len(plans)), float("nan"), dtype=torch.float64, device="cuda")
    best_ref = torch.full((n_sig,), -1, dtype=torch.int32, device="cuda")
    need = _lib.mci_averaged_error_workspace_size(len(plans), n_span, _lib.MCI_F32)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    _lib.mci_averaged_error(handles, a.data_ptr(), n_lo, n_span, n_sig, _lib.MCI_F32, eps_ref.data_ptr(),
                            best_ref.data_ptr(), ws.data_ptr(), need, stream)
    eps = torch.full((n_sig, len(plans)), float("nan"), dtype=torch.float64, device="cuda")
    best = torch.full((n_sig,), -1, dtype=torch.int32, device="cuda")
    _lib.mci_averaged_error_noalloc(handles, a.data_ptr(), n_lo, n_span, n_sig, _lib.MCI_F32, eps.data_ptr(),
                                    best.data_ptr(), stream)
    torch.cuda.synchronize()
    return eps.cpu().numpy(), best.cpu().numpy(), eps_ref.cpu().numpy(), best_ref.cpu().numpy()


def test_noalloc_matches_workspace_entry_point(torch_cuda):
    from paper_1802_10291_amd import Plan1D
    torch = torch_cuda
    rng = np.random.default_rng(2027)
    big = [Plan1D(N=N, n_out=2 * N * len(ch), channels=ch) for N, ch in
           [(4098, [("deriv", 0)]), (2049, [("deriv", 0), ("deriv", 1)]),
            (1366, [("deriv", 0), ("deriv", 1), ("deriv", 2)]), (2049, [("deriv", 0), ("hilbert", 0)]),
            (1025, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)])]]
    # first call: 5 plans, 300 signals x 16385 coefficients
    a1, lo1 = _spectra(rng, 300, 16385)
    eps, best, eps_ref, best_ref = _call_both(torch, big, a1, lo1)
    assert np.isfinite(eps_ref).all()
    assert np.array_equal(eps, eps_ref) and np.array_equal(best, best_ref)
    # second call: 2 plans, 7 signals x 3001 coefficients
    a2, lo2 = _spectra(rng, 7, 3001)
    eps, best, eps_ref, best_ref = _call_both(torch, big[1:3], a2, lo2)
    assert np.isfinite(eps_ref).all()
    assert np.array_equal(eps, eps_ref) and np.array_equal(best, best_ref)


def test_noalloc_rejects_sizes_beyond_the_static_array(torch_cuda):
    from paper_1802_10291_amd import MCIError, Plan1D, _lib
    torch = torch_cuda
    plans = [Plan1D(N=64, n_out=128, channels=[("deriv", 0)])] * 16
    n_span = 65533                       # 16 plans x 65533 FP32 weights + constants > 4 MiB
    a = torch.zeros((1, 8), dtype=torch.complex64, device="cuda")
    eps = torch.zeros((1, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(MCIError, match="INVALID_ARG"):
        _lib.mci_averaged_error_noalloc([p.handle for p in plans], a.data_ptr(), 0, n_span, 1, _lib.MCI_F32,
                                        eps.data_ptr(), 0, int(torch.cuda.current_stream().cuda_stream))
    assert _lib.mci_averaged_error_workspace_size(16, 65532, _lib.MCI_F32) <= 4 << 20
    assert _lib.mci_averaged_error_workspace_size(16, n_span, _lib.MCI_F32) > 4 << 20
