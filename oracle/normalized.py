"""Normalised adaptive filtering with a rotation field (line-integral convolution).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 8 (Application to Image Filtering) turns the extended convolution into a weighted
average: the output at p is the extended convolution of the signal divided by the
extended convolution of the constant signal 1 with the same field (eq. normalization),
so that every output is the sum of its neighbours' contributions over the sum of their
weights. For a field of rotations the filter keeps its integral, so the signal itself
is not rescaled (the normalised signal of the same section is needed only when the
field scales the filter). The line-integral-convolution visualisation of the same
section applies this to a noise image with a long, narrow anisotropic Gaussian whose
rotation at every pixel is the angle of a vector field; without the division the
result is the plain extended convolution.

Readings: zero boundary as everywhere else (the constant signal is 1 inside the image
and 0 outside, so the division also renormalises at the borders); the band-limited
filter of the decomposition is the filter (the paper band-limits before filtering).
"""
from __future__ import annotations

import numpy as np

from .extended import ext_conv_brute, ext_conv_fft, ext_conv_half


def normalized_conv_brute(H, theta, comps):
    """eq. (normalization) by the definition: both extended convolutions summed pixel by
    pixel (eq. Def-EConv). Returns (ratio, numerator, denominator), real parts."""
    H = np.asarray(H, dtype=np.float64)
    num = np.real(ext_conv_brute(H, theta, comps))
    den = np.real(ext_conv_brute(np.ones_like(H), theta, comps))
    return num / den, num, den


def normalized_conv_fft(H, theta, comps, P=None):
    """eq. (normalization) with both extended convolutions by the Sec. 4.1 route (full
    component stack k = -K..K)."""
    H = np.asarray(H, dtype=np.float64)
    num = np.real(ext_conv_fft(H, theta, comps, P))
    den = np.real(ext_conv_fft(np.ones_like(H), theta, comps, P))
    return num / den, num, den


def normalized_conv_half(H, alpha, comps_half, weights=None, P=None):
    """Real-filter form (components k = 0..K, weights 1, 2, ..., 2) of the same ratio."""
    H = np.asarray(H, dtype=np.float64)
    num = ext_conv_half(H, alpha, comps_half, weights, P)
    den = ext_conv_half(np.ones_like(H), alpha, comps_half, weights, P)
    return num / den, num, den
