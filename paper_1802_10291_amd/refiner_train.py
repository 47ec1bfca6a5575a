"""Training and evaluation of the residual refiner on pairs the method itself generates.

A pair is a synthetic high-resolution RGB image (random field + rectangles per colour
plane, see ``synth.images``), decimated by 2 (LR[i, j] = HR[2i, 2j]) and upsampled back by
separable MCI on the GPU (``Plan2D``); the refiner learns HR - MCI(LR).  After training, the
fallback bound tau is the 99.9th percentile of ||CNN(u)|| / ||u|| over the training pairs.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import Plan2D, Refiner, upsample_rgb


def _psnr(img: np.ndarray, ref: np.ndarray) -> float:
    mse = float(np.mean((np.clip(img, 0.0, 1.0) - ref) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def make_hr(first: int, count: int, size: int, seed_base: int, threads: int = 16) -> np.ndarray:
    """HR RGB images [count][3][size][size] float32, image i from seed seed_base + first + i."""
    from synth import images as SI
    out = np.empty((count, 3, size, size), dtype=np.float32)
    chunk = 32

    def work(c):
        n = min(chunk, count - c)
        out[c:c + n] = SI.rgb_images(first + c, n, size, size, seed_base=seed_base)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, range(0, count, chunk)))
    return out


def train(refiner: Refiner, n_pairs: int = 20000, batch: int = 16, size: int = 128, lr: float = 1e-3,
          epochs: int = 1, seed_base: int = 5_000_000, log=None):
    """Train on n_pairs method-generated pairs of size x size; returns the loss history."""
    import torch
    plan = Plan2D(size // 2, size // 2, 2)
    hist = []
    t0 = time.perf_counter()
    hr_all = make_hr(0, n_pairs, size, seed_base)
    if log:
        log(f"generated {n_pairs} pairs in {time.perf_counter() - t0:.1f} s")
    hr_dev = torch.from_numpy(hr_all).cuda()
    u_dev = torch.empty_like(hr_dev)
    for s in range(0, n_pairs, 256):
        e = min(n_pairs, s + 256)
        upsample_rgb(plan, hr_dev[s:e, :, ::2, ::2].contiguous(), out=u_dev[s:e])
    rng = np.random.default_rng(seed_base)
    step = 0
    total = epochs * (n_pairs // batch)
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n_pairs)).cuda()
        for s in range(0, n_pairs - batch + 1, batch):
            idx = order[s:s + batch]
            u = u_dev.index_select(0, idx)
            hr = hr_dev.index_select(0, idx)
            # cosine decay of the learning rate to 5% of its start
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * step / max(1, total))))
            loss = refiner.train_step(u, hr, float(lr_t))
            if step % 50 == 0:
                hist.append((step, float(loss)))
            step += 1
    torch.cuda.synchronize()
    # fallback bound: 99.9th percentile of the residual ratio over the training pairs
    ratios = []
    for s in range(0, n_pairs, 256):
        e = min(n_pairs, s + 256)
        _, r, _ = refiner.forward(u_dev[s:e])
        ratios.append(r.cpu().numpy())
    tau = float(np.quantile(np.concatenate(ratios), 0.999))
    p, _ = refiner.get_params()
    refiner.set_params(p, tau)
    if log:
        log(f"trained {step} steps in {time.perf_counter() - t0:.1f} s, tau = {tau:.4g}")
    return hist, tau


def evaluate(refiner: Refiner, n_images: int = 16, size: int = 512, seed_base: int = 6_000_000):
    """Mean PSNR (dB, clipped to [0, 1]) of plain MCI and of MCI + refiner on held-out images,
    and the fraction of images the refiner handled (the rest fell back)."""
    import torch
    hr = make_hr(0, n_images, size, seed_base)
    plan = Plan2D(size // 2, size // 2, 2)
    hr_dev = torch.from_numpy(hr).cuda()
    u = upsample_rgb(plan, hr_dev[:, :, ::2, ::2].contiguous())
    y, ratio, used = refiner.forward(u, fallback=True)
    u_h, y_h = u.cpu().numpy(), y.cpu().numpy()
    p_mci = float(np.mean([_psnr(u_h[i], hr[i]) for i in range(n_images)]))
    p_ref = float(np.mean([_psnr(y_h[i], hr[i]) for i in range(n_images)]))
    return p_mci, p_ref, float(used.float().mean())
