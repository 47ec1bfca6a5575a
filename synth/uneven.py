"""Seeded mixed workload of uneven instances: 1-D signals of many lengths and channel
counts plus 2-D images of many sizes, for the uneven-batch path.

Recipe (seed 4): 3584 one-dimensional instances with band length L drawn uniformly from
the 17 values {2^8 .. 2^16} and {3 2^7 .. 3 2^14}, M ~ U{2, 3, 4} derivative channels
(multipliers (i n)^m), N = ceil(L / M) samples per channel (the band M N >= L), n_out = 4 L
output points, and the batched workload's spectrum model (e^{-0.01 |n|} CN(0,1) plus 1e-3
white noise out to |n| = 2 L: not bandlimited); and 512 images with high-resolution side
drawn from {64, 96, ..., 1024} (2^k and 3 2^k), field images decimated by 2 and upsampled
back by 2 with M = 2 channels per axis.  The instance order is a seeded permutation.
The FP16-storage variant measures derivatives in units of N (channels (i n / N)^m).

Inputs are drawn per size class from a pool of distinct seeds (class c, pool entry k uses
seed 4_000_000 + 1000 c + k for signals, 4_500_000 + 1000 c + k for images); the pool
is tiled over the class's instances.  Nothing here is part of the reconstruction.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from .images import decimate, random_field_images
from .signals import smooth_noisy_batch

L_VALUES = [2 ** k for k in range(8, 17)] + [3 * 2 ** k for k in range(7, 15)]
SIDES_2D = [64, 96, 128, 192, 256, 384, 512, 768, 1024]


@dataclass(frozen=True)
class Instance:
    kind: str        # "1d" or "2d"
    L: int = 0       # 1-D band length asked for
    M: int = 0       # 1-D channels
    side: int = 0    # 2-D high-resolution side

    @property
    def N(self) -> int:
        return -(-self.L // self.M)

    @property
    def n_out(self) -> int:
        return 4 * self.L

    @property
    def lr_side(self) -> int:
        return self.side // 2

    def key(self) -> Tuple:
        return ("1d", self.L, self.M) if self.kind == "1d" else ("2d", self.side)


def instances(seed: int = 4, n1d: int = 3584, n2d: int = 512) -> List[Instance]:
    rng = np.random.default_rng(seed)
    Ls = rng.choice(L_VALUES, size=n1d)
    Ms = rng.integers(2, 5, size=n1d)
    sides = rng.choice(SIDES_2D, size=n2d)
    items = [Instance("1d", L=int(L), M=int(M)) for L, M in zip(Ls, Ms)]
    items += [Instance("2d", side=int(s)) for s in sides]
    order = rng.permutation(len(items))
    return [items[i] for i in order]


def classes(items: List[Instance]) -> Dict[Tuple, List[int]]:
    """Size class -> indices of its instances, classes in order of first appearance."""
    out: Dict[Tuple, List[int]] = {}
    for i, it in enumerate(items):
        out.setdefault(it.key(), []).append(i)
    return out


def class_pool(key: Tuple, class_id: int, count: int, dtype=np.float32, scaled: bool = False) -> np.ndarray:
    """`count` distinct inputs of one class: samples [count][M][N] or low-resolution
    images [count][side / 2][side / 2], rounded once to dtype.  scaled: derivative
    channels (i n / N)^m instead of (i n)^m (the FP16-storage variant; unscaled high
    derivatives leave FP16's range)."""
    if key[0] == "1d":
        _, L, M = key
        N = -(-L // M)
        return smooth_noisy_batch(0, count, M, N, 2 * L, seed_base=4_000_000 + 1000 * class_id, dtype=dtype,
                                  deriv_scale=float(N) if scaled else 1.0)
    side = key[1]
    hr = random_field_images(0, count, side, side, seed_base=4_500_000 + 1000 * class_id, dtype=np.float64)
    return decimate(hr, 2).astype(dtype)
