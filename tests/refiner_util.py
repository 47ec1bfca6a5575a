"""Helpers shared by the refiner tests: BF16 rounding and seeded parameter vectors."""
import numpy as np

from oracle import oracle as O

SL = O.CNN_SLICES


def bf16_round(x):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(O.CNN_NPARAM)
    p[SL["W1"]] = rng.standard_normal(32 * 27) * np.sqrt(2 / 27) * scale
    p[SL["W2"]] = rng.standard_normal(32 * 288) * np.sqrt(2 / 288) * scale
    p[SL["W3"]] = rng.standard_normal(32 * 288) * np.sqrt(2 / 288) * scale
    p[SL["W4"]] = rng.standard_normal(3 * 288) * 0.05 * scale
    for b in ("b1", "b2", "b3", "b4"):
        p[SL[b]] = rng.standard_normal(SL[b].stop - SL[b].start) * 0.05
    return p


def gpu_params(p):
    """The parameters the GPU computes with: FP32 biases, BF16-rounded weights."""
    q = p.astype(np.float32).copy()
    for w in ("W1", "W2", "W3", "W4"):
        q[SL[w]] = bf16_round(q[SL[w]])
    return q
