"""Seeded synthetic inputs for FFT multichannel interpolation.

This module only *makes inputs*: Fourier coefficients drawn from fixed seeds, the
channel samples g_m(t_p) = sum_n b_m(n) a(n) e^{i n t_p} of those signals, and
synthetic images.  It holds none of the reconstruction method's arithmetic, and both
the FP64 oracle and the GPU library receive exactly the arrays it returns (rounded
once to the storage type by the caller).
"""
from .signals import (  # noqa: F401
    trig_poly_real, sample_channels, deriv_multiplier, single_signal_fp64,
    smooth_noisy_spectrum, smooth_noisy_batch, random_bandlimited,
)
from .images import random_field_images, decimate, rgb_images  # noqa: F401
