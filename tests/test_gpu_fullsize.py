"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The oracle cannot reconstruct a whole benchmark batch in test time, so each workload runs
at full size on the GPU and is checked (1) against the oracle on sampled instances, and
(2) through properties that hold at any size: identical inputs tiled across the batch give
bit-identical outputs wherever they sit, and every output is finite.  Tolerances as in the
smaller parity tests, on relative L2 and on the element-wise error: 1e-5 for FP32 MCI; 1e-2 on the CNN residual of the refiner
against the oracle's BF16-operand mode (identical BF16-rounded operands).
"""
import numpy as np
import pytest

from oracle import oracle as O
from parity import worst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401  (fails loudly without the built library)
    return torch


def _rel(a, b):
    """Relative L2 and element-wise (max-abs over max |b|) error of one result: the larger."""
    return worst(a, b)


def test_batched_1d_full_batch(torch_cuda):
    """65536 signals x {f, f', f''} x 1366 samples -> 16384 points: the fused kernel over the
    whole batch, 6 sampled signals against the oracle, tiled copies bit-identical."""
    from paper_1802_10291_amd import Plan1D
    from synth import signals as S
    torch = torch_cuda
    B, M, N, n_out, pool = 65536, 3, 1366, 16384, 256
    host = S.smooth_noisy_batch(0, pool, M, N, 8192)
    g = torch.from_numpy(host).cuda().repeat(B // pool, 1, 1).contiguous()
    plan = Plan1D(N=N, n_out=n_out, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)], precision="f32")
    assert plan.info.path == 1
    y = plan.reconstruct(g)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    idx = [0, 257, 12345, 30000, 45678, 65535]
    ys = y[torch.tensor(idx, device="cuda")].cpu().numpy().astype(np.float64)
    ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
    want = O.reconstruct_1d(ch, host[[i % pool for i in idx]].astype(np.float64), n_out)
    for k in range(len(idx)):
        assert _rel(ys[k], want[k]) <= 1e-5, (idx[k], _rel(ys[k], want[k]))
    for i in (3, 100, 255):
        assert torch.equal(y[i], y[i + pool * 17]) and torch.equal(y[i], y[i + pool * 255])


@pytest.mark.parametrize("s,M,HR", [(2, 2, 512), (4, 2, 512), (3, 3, 384)])
def test_2d_full_batch(torch_cuda, s, M, HR):
    """256 images (x2: 256^2 -> 512^2, x4: 128^2 -> 512^2, x3 with three channels: 128^2 ->
    384^2) through the plan bench.py times, 2 sampled images against the oracle, tiled copies
    bit-identical."""
    from paper_1802_10291_amd import Plan2D
    from synth import images as SI
    torch = torch_cuda
    B, pool = 256, 8
    h = HR // s
    lr_host = SI.decimate(SI.random_field_images(0, pool, HR, HR), s)
    lr = torch.from_numpy(lr_host).cuda().repeat(B // pool, 1, 1).contiguous()
    plan = Plan2D(h, h, s, channels=M)
    out = plan.upsample(lr)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    for i in (1, 6):
        got = out[i + pool * 20].cpu().numpy().astype(np.float64)
        want = O.upsample_2d(lr_host[i].astype(np.float64), s, M)
        assert _rel(got, want) <= 1e-5, (i, _rel(got, want))
    for i in (0, 5):
        assert torch.equal(out[i], out[i + pool * 31])


def test_refiner_full_batch_crops(torch_cuda):
    """The refiner forward over 64 RGB images of 512^2 (the benchmark's batch).  Its receptive
    field is 9 x 9, so a 16 x 16 output window equals the oracle's output on the 24 x 24 crop
    around it (4-pixel halo, whose own zero padding never reaches the window); windows at the
    image corner check the zero padding of the full image."""
    from paper_1802_10291_amd import Refiner
    from refiner_util import bf16_round, gpu_params, random_params
    torch = torch_cuda
    B, H = 64, 512
    rng = np.random.default_rng(99)
    u = bf16_round(rng.uniform(size=(B, 3, H, H)).astype(np.float32)).reshape(B, 3, H, H)
    p = random_params(23)
    r = Refiner(seed=0)
    r.set_params(p.astype(np.float32))
    y, _, _ = r.forward(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    q = gpu_params(p).astype(np.float64)
    for b, y0, x0 in ((0, 200, 300), (37, 0, 0), (63, 496, 496), (12, 64, 480)):
        cy0, cx0 = max(0, y0 - 4), max(0, x0 - 4)
        cy1, cx1 = min(H, y0 + 20), min(H, x0 + 20)
        crop = u[b:b + 1, :, cy0:cy1, cx0:cx1].astype(np.float64)
        want = O.cnn_forward(q, crop, bf16=True)[0][:, y0 - cy0:y0 - cy0 + 16, x0 - cx0:x0 - cx0 + 16]
        got = y[b, :, y0:y0 + 16, x0:x0 + 16].cpu().numpy().astype(np.float64)
        base = u[b, :, y0:y0 + 16, x0:x0 + 16].astype(np.float64)
        assert _rel(got - base, want - base) <= 1e-2, (b, y0, x0, _rel(got - base, want - base))
