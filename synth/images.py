"""Seeded synthetic images standing in for natural-image test sets.

An image is a Gaussian random field whose power spectrum falls like 1/|k|^2 (DC
removed), min-max normalised to [0, 1], with K ~ U{0..20} axis-aligned rectangles of
uniform random intensity painted over it, clipped to [0, 1].  The low-resolution input
is the plain decimation LR[i, j] = HR[s i, s j].
"""
from __future__ import annotations

import numpy as np


def _one_image(rng: np.random.Generator, H: int, W: int, max_rects: int = 20) -> np.ndarray:
    ky = np.fft.fftfreq(H)[:, None] * H
    kx = np.fft.fftfreq(W)[None, :] * W
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    amp[k > 0] = 1.0 / k[k > 0]             # power ~ 1/|k|^2
    noise = rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))
    field = np.fft.ifft2(noise * amp).real
    lo, hi = field.min(), field.max()
    img = (field - lo) / (hi - lo) if hi > lo else np.zeros_like(field)
    n_rect = int(rng.integers(0, max_rects + 1))
    for _ in range(n_rect):
        y0, y1 = np.sort(rng.integers(0, H + 1, size=2))
        x0, x1 = np.sort(rng.integers(0, W + 1, size=2))
        img[y0:y1, x0:x1] = rng.uniform(0.0, 1.0)
    return np.clip(img, 0.0, 1.0)


def random_field_images(first: int, count: int, H: int = 512, W: int = 512, seed_base: int = 3_000_000,
                        dtype=np.float32) -> np.ndarray:
    """Images [count][H][W]; image i uses ``default_rng(seed_base + first + i)``."""
    out = np.empty((count, H, W), dtype=dtype)
    for i in range(count):
        out[i] = _one_image(np.random.default_rng(seed_base + first + i), H, W)
    return out


def rgb_images(first: int, count: int, H: int = 512, W: int = 512, seed_base: int = 5_000_000,
               dtype=np.float32) -> np.ndarray:
    """RGB images [count][3][H][W]; each colour plane is an independent field image."""
    out = np.empty((count, 3, H, W), dtype=dtype)
    for i in range(count):
        rng = np.random.default_rng(seed_base + first + i)
        for c in range(3):
            out[i, c] = _one_image(rng, H, W)
    return out


def decimate(hr: np.ndarray, s: int) -> np.ndarray:
    """LR[i, j] = HR[s i, s j] over the last two axes."""
    return np.ascontiguousarray(hr[..., ::s, ::s])
