"""Learned residual refiner y = u + CNN(u): the FP64 oracle (CPU pins) and the BF16-MFMA
GPU kernels against it.

The refiner is not in the paper, so nothing the paper prints pins it.  The oracle is pinned
by central differences of its own loss (gradient formulas), and by hand-built weights whose
output is known in closed form (tap orientation, zero padding, ReLU, the residual sum).

The oracle's BF16-operand mode (``bf16=True``: weights, the network input, every hidden
activation and every back-propagated gradient rounded to BF16 where the kernels store them,
FP64 arithmetic otherwise) is pinned against an independent PyTorch CPU autograd network in
FP64 with the same roundings, and its rounding against a bit-level FP32 -> BF16 rounding.

GPU tolerances.  Against the BF16-operand oracle the GPU sees identical rounded operands, so
what remains is FP32 accumulation (and the rare operand whose FP32 and FP64 values round to
neighbouring BF16 values): 1e-2 on the relative L2 and on the element-wise error of the CNN
residual and of each gradient tensor.  Against the plain FP64 oracle the BF16 storage itself
shows: three roundings of 2^-9 relative per hidden value give a few 1e-3 on the residual,
checked at 2e-2 (forward) and 5e-2 (gradients) as the error budget of BF16 storage.
"""
import numpy as np
import pytest

from oracle import oracle as O
from parity import worst
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


def test_oracle_bf16_rounding():
    """Round to nearest, ties to even, on hand-picked values, and equal to a bit-level FP32
    rounding (add half an ulp of BF16 plus the tie bit, truncate) on random FP32 values."""
    r = O.bf16_round
    assert r(1.0) == 1.0 and r(0.0) == 0.0
    assert r(1 + 2 ** -8) == 1.0                         # tie: even neighbour 1.0
    assert r(1 + 3 * 2 ** -8) == 1 + 2 ** -6             # tie: even neighbour 1 + 2/128
    assert r(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7      # just above the tie
    assert r(-(1 + 2 ** -8)) == -1.0
    assert r(3.0e-39) == bf16_round(np.float32(3.0e-39))  # FP32 subnormal range
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000)).astype(np.float32)
    want = bf16_round(x).astype(np.float64)
    got = np.array([r(float(v)) for v in x])
    assert np.array_equal(got, want)


def _torch_cnn(p, u, hr=None, bf16=False):
    """The same network in PyTorch CPU autograd, FP64, with the BF16 roundings as explicit
    steps: straight-through rounding of the stored forward operands and rounding hooks on
    the gradients that reach the stored activation gradients (after the ReLU masks) and the
    output gradient.  Returns y, or (loss, grad) when hr is given."""
    import torch
    F = torch.nn.functional
    rnd = (lambda t: t.detach().apply_(O.bf16_round)) if bf16 else (lambda t: t)

    class _R(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            return rnd(x.clone())

        @staticmethod
        def backward(ctx, g):
            return g

    R = _R.apply if bf16 else (lambda t: t)
    hook = (lambda t: t.register_hook(lambda g: rnd(g.clone()))) if bf16 else (lambda t: None)
    q = torch.tensor(p, dtype=torch.float64)
    layers, o = [], 0
    for cin, cout in ((3, 32), (32, 32), (32, 32), (32, 3)):
        w = q[o:o + cout * 9 * cin].view(cout, 3, 3, cin).permute(0, 3, 1, 2)
        o += cout * 9 * cin
        b = q[o:o + cout]
        o += cout
        layers.append((w, b))
    params = [t for wb in layers for t in wb]
    leaves = [t.detach().clone().requires_grad_(True) for t in params]
    ut = torch.tensor(u, dtype=torch.float64)
    x = R(ut)
    for i, (w, b) in enumerate(zip(leaves[0::2], leaves[1::2])):
        z = F.conv2d(x, R(w), b, padding=1)
        if i < 3:
            hook(z)                                  # gradient after the ReLU mask
            x = R(F.relu(z))
        else:
            hook(z)                                  # output gradient
            y = ut + z
    if hr is None:
        return y.detach().numpy()
    loss = ((y - torch.tensor(hr, dtype=torch.float64)) ** 2).mean()
    loss.backward()
    g = [leaves[2 * i].grad.permute(0, 2, 3, 1).reshape(-1) for i in range(4)]
    gb = [leaves[2 * i + 1].grad for i in range(4)]
    flat = torch.cat([t for pair in zip(g, gb) for t in pair]).numpy()
    return float(loss.detach()), flat


@pytest.mark.parametrize("bf16", [False, True])
def test_oracle_cnn_matches_torch_autograd(bf16):
    """The C oracle's forward, loss and parameter gradient equal a PyTorch CPU autograd
    network in FP64 (plain, and with the BF16 roundings as explicit steps)."""
    rng = np.random.default_rng(17 + bf16)
    p = random_params(9)
    u = rng.uniform(size=(2, 3, 9, 7))
    hr = rng.uniform(size=(2, 3, 9, 7))
    y = O.cnn_forward(p, u, bf16=bf16)
    assert np.abs(y - _torch_cnn(p, u, bf16=bf16)).max() <= 1e-12
    loss, g = O.cnn_grad(p, u, hr, bf16=bf16)
    lt, gt = _torch_cnn(p, u, hr, bf16=bf16)
    assert abs(loss - lt) <= 1e-13 * lt
    for name, s in SL.items():
        assert np.abs(g[s] - gt[s]).max() <= 1e-12 * max(np.abs(gt[s]).max(), 1e-30), name
    if bf16:   # the roundings matter: the two modes differ by about the BF16 spacing
        d = worst(O.cnn_forward(p, u, bf16=True) - u, O.cnn_forward(p, u) - u)
        assert 1e-4 < d < 3e-2, d


def test_oracle_cnn_hand_built_weights_bf16():
    """The hand-built network of the test above in BF16-operand mode: the input and each
    hidden activation round where stored, so the closed form takes the same roundings."""
    p = np.zeros(O.CNN_NPARAM)
    W1 = p[SL["W1"]].reshape(32, 9, 3)
    W1[0, 2, 1] = 1.0
    p[SL["b1"]][0] = 0.25 + 2 ** -12                     # makes a1 need rounding
    W3 = p[SL["W3"]].reshape(32, 9, 32)
    W2 = p[SL["W2"]].reshape(32, 9, 32)
    W2[0, 4, 0] = 1.0
    W3[0, 4, 0] = 3.0
    W4 = p[SL["W4"]].reshape(3, 9, 32)
    W4[2, 4, 0] = 0.5
    rng = np.random.default_rng(6)
    u = rng.uniform(0.0, 1.0, size=(1, 3, 6, 7))
    x = bf16_round(u).astype(np.float64)
    shifted = np.zeros((6, 7))
    shifted[1:, :-1] = x[0, 1, :-1, 1:]
    a1 = bf16_round(np.maximum(shifted + p[SL["b1"]][0], 0.0)).astype(np.float64)
    a3 = bf16_round(3.0 * a1).astype(np.float64)
    want = u.copy()
    want[0, 2] += 0.5 * a3
    assert np.abs(O.cnn_forward(p, u, bf16=True) - want).max() < 1e-14
    assert np.abs(O.cnn_forward(p, u, bf16=True) - O.cnn_forward(p, u)).max() > 1e-4


# ------------------------------------------------------------------ GPU
@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_10291_amd  # noqa: F401
    return torch


def rel(a, b):
    """Relative L2 and element-wise (max-abs over max |b|) error: the larger."""
    return worst(a, b)


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
    q = gpu_params(p).astype(np.float64)
    want = O.cnn_forward(q, u.astype(np.float64), bf16=True)
    err = rel(y - u, want - u)
    print(f"refiner forward vs BF16-operand oracle: {err:.3e}")
    assert err <= 1e-2
    assert rel(y - u, O.cnn_forward(q, u.astype(np.float64)) - u) <= 2e-2     # BF16 storage budget
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
    q = gpu_params(p).astype(np.float64)
    lw, gw = O.cnn_grad(q, u.astype(np.float64), hr.astype(np.float64), bf16=True)
    assert loss == pytest.approx(lw, rel=1e-2)
    for name, s in SL.items():
        err = rel(g[s], gw[s])
        print(f"refiner gradient {name} vs BF16-operand oracle: {err:.3e}")
        assert err <= 1e-2, (name, err)
    l64, g64 = O.cnn_grad(q, u.astype(np.float64), hr.astype(np.float64))     # BF16 storage budget
    assert loss == pytest.approx(l64, rel=2e-2)
    for name, s in SL.items():
        assert rel(g[s], g64[s]) <= 5e-2, (name, rel(g[s], g64[s]))


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
    """The inference forward (with the ratio's per-tile sums in its last epilogue, and layers
    2 and 3 in one pass) and the forward inside a training step (layer by layer) compute the
    same values, so the training loss equals the squared error of the inference output (up
    to the order of the loss reduction), on tiled and ragged image sizes."""
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


@pytest.mark.gpu
@pytest.mark.parametrize("B,H,W", [(2, 32, 48), (3, 37, 50), (1, 5, 7), (2, 16, 16), (2, 512, 512)])
def test_two_layer_pass_equals_layered_forward(torch_cuda, monkeypatch, B, H, W):
    """The inference pass that runs layers 2 and 3 in one kernel (layer 2 on the 18 x 18
    region of each tile, its BF16 result kept on chip) accumulates every output in the same
    order as the layer-by-layer kernels and rounds the intermediate the same way: the outputs
    and ratios are bit-identical, on ragged sizes, an image smaller than one tile and the
    benchmark's 512 x 512."""
    from paper_1802_10291_amd import Refiner
    torch = torch_cuda
    rng = np.random.default_rng(B * H * W)
    r = Refiner(seed=4)
    r.set_params(random_params(23).astype(np.float32))
    u = torch.from_numpy(rng.uniform(size=(B, 3, H, W)).astype(np.float32)).cuda()
    monkeypatch.delenv("MCI_REFINER_LAYERED", raising=False)
    y1, ratio1, _ = r.forward(u)
    y1 = y1.clone()
    monkeypatch.setenv("MCI_REFINER_LAYERED", "1")
    y2, ratio2, _ = r.forward(u)
    assert torch.equal(y1, y2)
    assert torch.equal(ratio1, ratio2)
    assert (y1 - u).abs().max().item() > 0      # the network changed the image


def test_training_images_recipe_on_cpu():
    """The refiner's pair generator (run here on the CPU device): values in [0, 1], seeded and
    repeatable, different seeds give different images, and painted rectangles show as
    constant blocks."""
    import torch
    from paper_1802_10291_amd.refiner_train import gpu_rgb_images
    a = gpu_rgb_images([11, 12], 64, device="cpu")
    b = gpu_rgb_images([11, 12], 64, device="cpu")
    assert a.shape == (2, 3, 64, 64) and a.dtype == torch.float32
    assert torch.equal(a, b) and not torch.equal(a[0], a[1])
    assert float(a.min()) >= 0.0 and float(a.max()) <= 1.0
    # some plane has a run of equal values from a rectangle (K ~ U{0..20} per plane)
    runs = (a[..., 1:] == a[..., :-1]).float().mean()
    assert float(runs) > 0.05


@pytest.mark.gpu
def test_checkpoint_resume_is_bit_identical(torch_cuda, tmp_path):
    """Training stopped at a checkpoint and resumed in a fresh refiner (other initial
    weights) continues bit for bit: the same parameters after the same further steps, across
    an epoch boundary.  The checkpoint bytes round-trip, and a foreign buffer is refused."""
    from paper_1802_10291_amd import MCIError, Refiner
    from paper_1802_10291_amd.refiner_train import Trainer
    r1 = Refiner(seed=4)
    t1 = Trainer(r1, n_pairs=64, batch=8, size=64, lr=2e-3, epochs=2)
    t1.run(max_steps=5)
    path = str(tmp_path / "ck.npz")
    t1.save(path)
    t1.run(max_steps=7)                       # steps 5..11 cross the epoch boundary at 8
    p1, _ = r1.get_params()
    r2 = Refiner(seed=99)
    t2 = Trainer(r2, n_pairs=64, batch=8, size=64, lr=2e-3, epochs=2)
    t2.load(path)
    assert (t2.epoch, t2.pos, t2.step) == (0, 40, 5)
    t2.run(max_steps=7)
    p2, _ = r2.get_params()
    assert np.array_equal(p1, p2)
    s1 = r1.save_state()
    r3 = Refiner(seed=7)
    r3.load_state(s1)
    assert r3.save_state() == s1
    with pytest.raises(MCIError):
        r3.load_state(b"\0" * len(s1))
    with pytest.raises(ValueError):
        Trainer(r3, n_pairs=64, batch=8, size=64, lr=1e-3, epochs=2).load(path)
