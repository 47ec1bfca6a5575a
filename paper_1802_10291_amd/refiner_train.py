"""Training and evaluation of the residual refiner on pairs the method itself generates.

A pair is a synthetic high-resolution RGB image, decimated by 2 (LR[i, j] = HR[2i, 2j]) and
upsampled back by separable MCI on the GPU (``Plan2D``); the refiner learns HR - MCI(LR).
After training, the fallback bound tau is the 99.9th percentile of ||CNN(u)|| / ||u|| over
the training pairs.

The images are made on the GPU, batch by batch, so that pairs of 512 x 512 need no host
generation or storage: each colour plane is a Gaussian random field whose power falls like
1/|k|^2 (DC removed), min-max normalised to [0, 1], with K ~ U{0..20} axis-aligned
rectangles of uniform random intensity painted over it in order and the result clipped to
[0, 1] -- the recipe of ``synth.images`` -- drawn from a torch generator seeded with the
pair's seed (seed_base + pair index).  Epoch e visits the pairs in the order of
``numpy.random.default_rng(seed_base + e).permutation``, so the position (epoch, offset,
step) and the refiner's state determine the rest of a run: a checkpoint holds exactly that.
"""
from __future__ import annotations

import time

import numpy as np

from . import Plan2D, Refiner, upsample_rgb

MAX_RECTS = 20


def gpu_rgb_images(seeds, size: int, device: str = "cuda"):
    """HR RGB images [len(seeds)][3][size][size] float32 on the GPU, image i from seeds[i]."""
    import torch
    n = len(seeds)
    noise = torch.empty((n, 3, size, size, 2), dtype=torch.float32, device=device)
    K = torch.empty((n, 3), dtype=torch.int64, device=device)
    corners = torch.empty((n, 3, MAX_RECTS, 4), dtype=torch.int64, device=device)
    inten = torch.empty((n, 3, MAX_RECTS), dtype=torch.float32, device=device)
    for i, sd in enumerate(seeds):
        g = torch.Generator(device=device)
        g.manual_seed(int(sd))
        noise[i] = torch.randn((3, size, size, 2), generator=g, device=device)
        K[i] = torch.randint(0, MAX_RECTS + 1, (3,), generator=g, device=device)
        corners[i] = torch.randint(0, size + 1, (3, MAX_RECTS, 4), generator=g, device=device)
        inten[i] = torch.rand((3, MAX_RECTS), generator=g, device=device)
    f = torch.fft.fftfreq(size, device=device) * size
    k = torch.sqrt(f[:, None] ** 2 + f[None, :] ** 2)
    amp = torch.where(k > 0, 1.0 / torch.clamp(k, min=1e-30), torch.zeros_like(k))
    field = torch.fft.ifft2(torch.view_as_complex(noise) * amp).real
    lo = field.amin(dim=(-2, -1), keepdim=True)
    hi = field.amax(dim=(-2, -1), keepdim=True)
    img = torch.where(hi > lo, (field - lo) / torch.clamp(hi - lo, min=1e-30), torch.zeros_like(field))
    # rectangles in order: the last one covering a pixel sets it
    y0 = torch.minimum(corners[..., 0], corners[..., 1])
    y1 = torch.maximum(corners[..., 0], corners[..., 1])
    x0 = torch.minimum(corners[..., 2], corners[..., 3])
    x1 = torch.maximum(corners[..., 2], corners[..., 3])
    pos = torch.arange(size, device=device)
    top = torch.zeros((n, 3, size, size), dtype=torch.int64, device=device)
    for r in range(MAX_RECTS):
        on = (r < K)[..., None, None]
        rows = (pos >= y0[..., r, None]) & (pos < y1[..., r, None])
        cols = (pos >= x0[..., r, None]) & (pos < x1[..., r, None])
        inside = rows[..., :, None] & cols[..., None, :] & on
        top = torch.where(inside, torch.full_like(top, r + 1), top)
    painted = torch.gather(torch.cat([torch.zeros((n, 3, 1), device=device), inten], dim=2), 2,
                           top.view(n, 3, -1)).view(n, 3, size, size)
    img = torch.where(top > 0, painted, img)
    return torch.clamp(img, 0.0, 1.0).contiguous()


class Trainer:
    """Adam training of a refiner on method-generated pairs, resumable from a checkpoint."""

    def __init__(self, refiner: Refiner, n_pairs: int = 20000, batch: int = 16, size: int = 128, lr: float = 1e-3,
                 epochs: int = 1, seed_base: int = 5_000_000):
        self.r, self.n_pairs, self.batch, self.size = refiner, int(n_pairs), int(batch), int(size)
        self.lr, self.epochs, self.seed_base = float(lr), int(epochs), int(seed_base)
        self.plan = Plan2D(size // 2, size // 2, 2)
        self.epoch = self.pos = self.step = 0
        self.per_epoch = self.n_pairs // self.batch
        self.total = self.epochs * self.per_epoch

    def _order(self, epoch: int) -> np.ndarray:
        return np.random.default_rng(self.seed_base + epoch).permutation(self.n_pairs)

    def pairs(self, idx):
        """(u, hr) on the GPU for pair indices idx: HR images and their MCI upsamples."""
        hr = gpu_rgb_images([self.seed_base + int(i) for i in idx], self.size)
        u = upsample_rgb(self.plan, hr[:, :, ::2, ::2].contiguous())
        return u, hr

    def done(self) -> bool:
        return self.step >= self.total

    def run(self, max_steps=None, log_every: int = 50):
        """Train until the schedule ends (or max_steps more steps); returns [(step, loss)]."""
        hist = []
        stop = self.total if max_steps is None else min(self.total, self.step + int(max_steps))
        order = self._order(self.epoch)
        while self.step < stop:
            idx = order[self.pos:self.pos + self.batch]
            u, hr = self.pairs(idx)
            # cosine decay of the learning rate to 5% of its start
            lr_t = self.lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * self.step / max(1, self.total))))
            loss = self.r.train_step(u, hr, float(lr_t))
            if self.step % log_every == 0:
                hist.append((self.step, float(loss)))
            self.step += 1
            self.pos += self.batch
            if self.pos + self.batch > self.n_pairs:
                self.epoch += 1
                self.pos = 0
                order = self._order(self.epoch)
        return hist

    def fallback_bound(self, chunk: int = 64) -> float:
        """tau = the 99.9th percentile of ||CNN(u)|| / ||u|| over the training pairs; set on the refiner."""
        ratios = []
        for s in range(0, self.n_pairs, chunk):
            u, _ = self.pairs(range(s, min(self.n_pairs, s + chunk)))
            _, r, _ = self.r.forward(u)
            ratios.append(r.cpu().numpy())
        tau = float(np.quantile(np.concatenate(ratios), 0.999))
        p, _ = self.r.get_params()
        self.r.set_params(p, tau)
        return tau

    def save(self, path: str) -> None:
        """Checkpoint: the refiner's training state and the position in the schedule."""
        meta = np.array([self.epoch, self.pos, self.step, self.n_pairs, self.batch, self.size, self.epochs,
                         self.seed_base], dtype=np.int64)
        np.savez(path, state=np.frombuffer(self.r.save_state(), dtype=np.uint8), meta=meta,
                 lr=np.array([self.lr], dtype=np.float64))

    def load(self, path: str) -> None:
        with np.load(path, allow_pickle=False) as z:
            meta = z["meta"].tolist()
            if meta[3:] != [self.n_pairs, self.batch, self.size, self.epochs, self.seed_base] or \
                    float(z["lr"][0]) != self.lr:
                raise ValueError("checkpoint of another training schedule")
            self.r.load_state(z["state"].tobytes())
            self.epoch, self.pos, self.step = meta[:3]


def train(refiner: Refiner, n_pairs: int = 20000, batch: int = 16, size: int = 128, lr: float = 1e-3,
          epochs: int = 1, seed_base: int = 5_000_000, log=None):
    """Train on n_pairs method-generated pairs of size x size; returns (loss history, tau)."""
    import torch
    t0 = time.perf_counter()
    tr = Trainer(refiner, n_pairs, batch, size, lr, epochs, seed_base)
    hist = tr.run()
    torch.cuda.synchronize()
    tau = tr.fallback_bound()
    if log:
        log(f"trained {tr.step} steps on {n_pairs} pairs of {size}^2 in {time.perf_counter() - t0:.1f} s, "
            f"tau = {tau:.4g}")
    return hist, tau


def evaluate(refiner: Refiner, n_images: int = 16, size: int = 512, seed_base: int = 6_000_000, chunk: int = 32):
    """Mean PSNR (dB, clipped to [0, 1]) of plain MCI and of MCI + refiner on held-out images,
    and the fraction of images the refiner handled (the rest fell back)."""
    import torch
    plan = Plan2D(size // 2, size // 2, 2)
    p_mci, p_ref, used_n = [], [], 0
    for s in range(0, n_images, chunk):
        hr = gpu_rgb_images([seed_base + i for i in range(s, min(n_images, s + chunk))], size)
        u = upsample_rgb(plan, hr[:, :, ::2, ::2].contiguous())
        y, _, used = refiner.forward(u, fallback=True)
        for img, out in ((u, p_mci), (y, p_ref)):
            mse = ((torch.clamp(img, 0.0, 1.0).double() - hr.double()) ** 2).mean(dim=(1, 2, 3))
            out.extend((10.0 * torch.log10(1.0 / mse)).cpu().tolist())
        used_n += int(used.sum())
    return float(np.mean(p_mci)), float(np.mean(p_ref)), used_n / n_images
