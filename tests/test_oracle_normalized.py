"""Pins of the oracle's normalised filtering with a rotation field (Sec. 8, eq.
normalization; line-integral convolution). CPU only."""
import numpy as np
import pytest
import scipy.signal as ss

import oracle as O
from synthetic import anisotropic_gaussian, blurred_noise, theta_field, vortex_field


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def lic_case():
    H = np.random.default_rng(3).random((23, 26))
    th = vortex_field((23, 26), 4, sigma=3.0).astype(np.float64)
    comps, _ = O.angular_components(anisotropic_gaussian(11, 3.0, 1.0), 5)
    return H, th, comps


def test_brute_fft_and_half_forms_agree(lic_case):
    H, th, comps = lic_case
    yb, nb, db = O.normalized_conv_brute(H, th, comps)
    yf, nf, df = O.normalized_conv_fft(H, th, comps)
    yh, nh, dh = O.normalized_conv_half(H, th, O.half_components(comps))
    assert rel(nf, nb) < 1e-12 and rel(df, db) < 1e-12 and rel(yf, yb) < 1e-12
    assert rel(yh, yb) < 1e-12 and rel(dh, db) < 1e-12


def test_constant_signal_is_returned_unchanged(lic_case):
    """The output is a weighted average of the neighbours: a constant image maps to itself
    under any field, at the borders too (the constant signal is zero outside the image)."""
    _, th, comps = lic_case
    c = 0.37
    y, _, den = O.normalized_conv_brute(np.full(th.shape, c), th, comps)
    assert np.min(den) > 0.1
    assert np.max(np.abs(y - c)) < 1e-13


def test_constant_field_is_textbook_normalised_convolution(lic_case):
    """At a constant angle both convolutions are plain convolutions with the rotated
    band-limited filter (scipy.signal.convolve2d, zero fill)."""
    H, _, comps = lic_case
    for t0 in (0.0, 1.1, 3.7):
        Ft = np.real(O.rotated_filter(comps, t0))
        th = np.full(H.shape, t0)
        y, num, den = O.normalized_conv_brute(H, th, comps)
        rn = ss.convolve2d(H, Ft, mode="same", boundary="fill")
        rd = ss.convolve2d(np.ones_like(H), Ft, mode="same", boundary="fill")
        assert rel(num, rn) < 1e-12 and rel(den, rd) < 1e-12 and rel(y, rn / rd) < 1e-12


def test_no_division_is_the_extended_convolution(lic_case):
    H, th, comps = lic_case
    _, num, _ = O.normalized_conv_fft(H, th, comps)
    assert rel(num, np.real(O.ext_conv_brute(H, th, comps))) < 1e-12


def test_quarter_turn_equivariance():
    """Rotating image and field by 90 degrees on the grid (field shifted by -pi/2)
    rotates the normalised output the same way, exactly."""
    n = 18
    H = blurred_noise((n, n), 21).astype(np.float64)
    th = theta_field((n, n), 22).astype(np.float64)
    comps, _ = O.angular_components(anisotropic_gaussian(9, 3.0, 1.0), 4)
    a, _, _ = O.normalized_conv_brute(np.rot90(H), np.rot90(th) - np.pi / 2, comps)
    b, _, _ = O.normalized_conv_brute(H, th, comps)
    assert rel(a, np.rot90(b)) < 1e-13


def test_smoothing_follows_the_field():
    """Noise smoothed along a horizontal field varies less along rows than along columns
    (the filter's long axis lies along x at angle 0), and the other way at pi/2."""
    H = np.random.default_rng(7).random((40, 40))
    comps, _ = O.angular_components(anisotropic_gaussian(15, 5.0, 0.8), 8)
    for t0, along_rows in ((0.0, True), (np.pi / 2, False)):
        y, _, _ = O.normalized_conv_half(H, np.full(H.shape, t0), O.half_components(comps))
        c = y[8:-8, 8:-8]
        dr = np.mean(np.abs(np.diff(c, axis=1)))   # along a row (x)
        dc = np.mean(np.abs(np.diff(c, axis=0)))   # along a column (y)
        assert (dr < 0.5 * dc) if along_rows else (dc < 0.5 * dr)
