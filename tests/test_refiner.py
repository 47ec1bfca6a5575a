"""Learned residual refiner y = u + CNN(u): the FP64 oracle (CPU pins) and the BF16-MFMA
GPU kernels against it.

The refiner is not in the paper, so nothing the paper prints pins it.  The oracle is pinned
by central differences of its own loss (gradient formulas), and by hand-built weights whose
output is known in closed form (tap orientation, zero padding, ReLU, the residual sum).

GPU tolerances.  The GPU rounds weights and the input to BF16 (the oracle gets the same
rounded values) and also stores every hidden activation and back-propagated gradient in
BF16 (relative rounding 2^-9 = 2e-3 per value).  Through three such roundings the relative L2
error of the CNN residual is a few 1e-3: forward tolerance 2e-2, gradients 5e-2 per tensor.
"""
import numpy as np
import pytest

from oracle import oracle as O
from refiner_util import bf16_round, gpu_params, random_params

SL = O.CNN_SLICES


# ------------------------------------------------------------------ oracle pins (CPU)
def test_oracle_cnn_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = random_params(2, 0.7)
    u = rng.uniform(size=(2, 3, 7, 6))
    hr = rng.uniform(size=(2, 3, 7, 6))
    _, g = O.cnn_grad(p, u, hr)
    idx = np.concatenate([rng.choice(np.arange(s.start, s.stop), min(6, s.stop - s.start), replace=False)
                          for s in SL.values()])
    for i in idx:
        h = 1e-6
        pp = p.copy(); pp[i] += h
        lp, _ = O.cnn_grad(pp, u, hr)
        pp[i] -= 2 * h
        lm, _ = O.cnn_grad(pp, u, hr)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_oracle_cnn_zero_last_layer_is_identity():
    rng = np.random.default_rng(3)
    p = random_params(4)
    p[SL["W4"]] = 0.0
    p[SL["b4"]] = 0.0
    u = rng.uniform(size=(1, 3, 5, 9))
    assert np.array_equal(O.cnn_forward(p, u), u)


def test_oracle_cnn_hand_built_weights():
    """Channel 0 of layer 1 reads input channel 1 at tap (dy, dx) = (0, 2), i.e. pixel
    (y - 1, x + 1) with zero padding; layers 2-3 pass channel 0 through; layer 4 adds
    0.5 * it to output channel 2.  Biases shift by known amounts through the ReLUs."""
    p = np.zeros(O.CNN_NPARAM)
    W1 = p[SL["W1"]].reshape(32, 9, 3)
    W1[0, 0 * 3 + 2, 1] = 1.0
    p[SL["b1"]][0] = 0.25
    W2 = p[SL["W2"]].reshape(32, 9, 32)
    W2[0, 4, 0] = 1.0
    W3 = p[SL["W3"]].reshape(32, 9, 32)
    W3[0, 4, 0] = 2.0
    p[SL["b3"]][0] = -0.5
    W4 = p[SL["W4"]].reshape(3, 9, 32)
    W4[2, 4, 0] = 0.5
    p[SL["b4"]][1] = 0.125
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, size=(1, 3, 6, 7))
    shifted = np.zeros((6, 7))
    shifted[1:, :-1] = u[0, 1, :-1, 1:]                  # value at (y - 1, x + 1)
    a1 = np.maximum(shifted + 0.25, 0.0)
    a3 = np.maximum(2.0 * a1 - 0.5, 0.0)
    want = u.copy()
    want[0, 2] += 0.5 * a3
    want[0, 1] += 0.125
    assert np.abs(O.cnn_forward(p, u) - want).max() < 1e-14


# ------------------------------------------------------------------ GPU
@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401
    return torch


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.gpu
@pytest.mark.parametrize("H,W", [(32, 48), (20, 37)])
def test_refiner_forward_parity(torch_cuda, H, W):
    from paper_1802_10291_amd import Refiner
    rng = np.random.default_rng(H + W)
    p = random_params(7)
    u = bf16_round(rng.uniform(size=(2, 3, H, W))).reshape(2, 3, H, W)
    r = Refiner(seed=0)
    r.set_params(p.astype(np.float32))
    y, ratio, used = r.forward(torch_cuda.from_numpy(u).cuda())
    y = y.cpu().numpy().astype(np.float64)
    want = O.cnn_forward(gpu_params(p).astype(np.float64), u.astype(np.float64))
    assert rel(y - u, want - u) <= 2e-2
    # ratio = ||y - u|| / ||u|| per image
    rr = [np.linalg.norm(y[b] - u[b]) / np.linalg.norm(u[b]) for b in range(2)]
    assert np.allclose(ratio.cpu().numpy(), rr, rtol=1e-4)


@pytest.mark.gpu
def test_refiner_gradient_parity(torch_cuda):
    from paper_1802_10291_amd import Refiner
    rng = np.random.default_rng(11)
    p = random_params(12)
    H, W = 32, 40
    u = bf16_round(rng.uniform(size=(2, 3, H, W))).reshape(2, 3, H, W)
    hr = rng.uniform(size=(2, 3, H, W)).astype(np.float32)
    r = Refiner(seed=0)
    r.set_params(p.astype(np.float32))
    loss = float(r.backward(torch_cuda.from_numpy(u).cuda(), torch_cuda.from_numpy(hr).cuda()))
    g = r.get_grads().astype(np.float64)
    lw, gw = O.cnn_grad(gpu_params(p).astype(np.float64), u.astype(np.float64), hr.astype(np.float64))
    assert loss == pytest.approx(lw, rel=2e-2)
    for name, s in SL.items():
        assert rel(g[s], gw[s]) <= 5e-2, (name, rel(g[s], gw[s]))


@pytest.mark.gpu
def test_refiner_fallback(torch_cuda):
    from paper_1802_10291_amd import Refiner
    rng = np.random.default_rng(13)
    u = torch_cuda.from_numpy(rng.uniform(size=(3, 3, 16, 16)).astype(np.float32)).cuda()
    r = Refiner(seed=1)
    p, _ = r.get_params()
    p[SL["b4"]] = 0.3                      # a large residual on every image
    r.set_params(p, tau=0.0)               # bound 0: every image falls back
    y, ratio, used = r.forward(u, fallback=True)
    assert used.cpu().numpy().tolist() == [0, 0, 0]
    assert torch_cuda.equal(y, u)
    r.set_params(p, tau=1e9)               # no image falls back
    y, ratio, used = r.forward(u, fallback=True)
    assert used.cpu().numpy().tolist() == [1, 1, 1]
    assert not torch_cuda.equal(y, u)
    p[SL["W4"]] = np.nan                   # broken weights: NaN ratio falls back
    r.set_params(p, tau=1e9)
    y, ratio, used = r.forward(u, fallback=True)
    assert used.cpu().numpy().tolist() == [0, 0, 0] and torch_cuda.equal(y, u)


@pytest.mark.gpu
def test_refiner_params_roundtrip(torch_cuda):
    from paper_1802_10291_amd import Refiner
    r = Refiner(seed=5)
    p, tau = r.get_params()
    assert p.size == O.CNN_NPARAM and tau == 0.0
    q = p * 2
    r.set_params(q, tau=0.25)
    p2, tau2 = r.get_params()
    assert np.array_equal(p2, q) and tau2 == pytest.approx(0.25)


@pytest.mark.gpu
def test_refiner_training_beats_plain_mci(torch_cuda):
    """Trained on pairs the method generates (HR -> decimate -> MCI), the refiner raises the
    PSNR of held-out upsamples over plain MCI; training is deterministic."""
    from paper_1802_10291_amd import Refiner
    from paper_1802_10291_amd import refiner_train as RT
    r = Refiner(seed=0)
    hist, tau = RT.train(r, n_pairs=2048, batch=16, size=128, lr=1e-3, epochs=2)
    assert hist[-1][1] < hist[0][1]
    p_mci, p_ref, frac = RT.evaluate(r, n_images=8, size=256)
    print(f"PSNR MCI {p_mci:.3f} dB, refined {p_ref:.3f} dB")
    assert frac == 1.0 and tau > 0
    assert p_ref > p_mci


@pytest.mark.gpu
@pytest.mark.parametrize("H,W", [(64, 48), (37, 50)])
def test_forward_output_matches_training_loss(torch_cuda, H, W):
    """The inference forward (with the ratio's per-tile sums in its last epilogue) and the
    forward inside a training step run the same layer kernels, so the training loss equals
    the squared error of the inference output (up to the order of the loss reduction), on
    tiled and ragged image sizes."""
    from paper_1802_10291_amd import Refiner
    torch = torch_cuda
    rng = np.random.default_rng(H * W)
    r = Refiner(seed=3)
    r.set_params(random_params(19).astype(np.float32))
    u = torch.from_numpy(rng.uniform(size=(3, 3, H, W)).astype(np.float32)).cuda()
    hr = torch.from_numpy(rng.uniform(size=(3, 3, H, W)).astype(np.float32)).cuda()
    y, _, _ = r.forward(u)
    loss = float(r.backward(u, hr))
    want = float(((y.double() - hr.double()) ** 2).mean())
    assert loss == pytest.approx(want, rel=1e-5)
