"""Pins of the oracle's scale-group smoothing and its analytic gradients. CPU only."""
import numpy as np
import pytest
import scipy.signal as ss

import oracle as O
from synthetic import blurred_noise, random_filter, theta_field, scale_field


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


SMALL = O.ScaleParams(sigma0=1.0, s_min=1.0, s_max=2.0, n_comp=12, period_factor=1.5)


def test_scale_trig_interpolation_hits_samples():
    """The component sum reproduces h at its sample points (DFT inversion, Nyquist as
    cosine), so at s = 1 the band-limited filter equals g wherever ln|x| is a sample."""
    p = SMALL
    ks, c = O.scale.scale_coefficients(p)
    n = p.n_comp
    for j in range(n):
        u = p.u_lo + j * p.L / n
        val = 0.0
        for k, ck in zip(ks, c):
            w = 2 * np.pi * k / p.L
            val += np.real(ck) * np.cos(w * (u - p.u_lo)) if k == -(n // 2) else np.real(ck * np.exp(1j * w * (u - p.u_lo)))
        assert val == pytest.approx(float(O.scale._h(u, p)), abs=1e-13)


def test_scale_brute_equals_component_route():
    H = blurred_noise((20, 17), 30).astype(np.float64)
    s = scale_field((20, 17), 31, 1.0, 2.0, sigma=3.0).astype(np.float64)
    yb, nb, db = O.scale_smooth_brute(H, s, SMALL)
    yf, nf, df = O.scale_smooth_fft(H, s, SMALL)
    assert rel(nf, nb) < 1e-12 and rel(df, db) < 1e-12 and rel(yf, yb) < 1e-12


def test_scale_ratio_preserves_constants():
    """eq. (normalization): a constant signal is returned unchanged whatever the field."""
    s = scale_field((18, 18), 32, 1.0, 2.0, sigma=3.0).astype(np.float64)
    y, _, _ = O.scale_smooth_fft(np.full((18, 18), 0.37), s, SMALL)
    assert np.max(np.abs(y - 0.37)) < 1e-13


def test_constant_scale_is_textbook_convolution():
    H = blurred_noise((19, 23), 33).astype(np.float64)
    s0 = 1.6
    s = np.full(H.shape, s0)
    Fs = O.scale_filter_at(SMALL, s0)
    ref_num = ss.convolve2d(H / s0 ** 2, Fs, mode="same")
    ref_den = ss.convolve2d(np.full(H.shape, 1 / s0 ** 2), Fs, mode="same")
    y, num, den = O.scale_smooth_fft(H, s, SMALL)
    assert rel(num, ref_num) < 1e-12 and rel(den, ref_den) < 1e-12
    assert rel(y, ref_num / ref_den) < 1e-12


def test_scaled_filter_approximates_gaussian():
    """The 24-component reading approximates g(|x|/s) (approximation error, not parity)."""
    p = O.ScaleParams()
    R = p.R
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    r = np.hypot(xx, yy)
    for s in (1.0, 2.5, 8.0):
        exact = np.where(r <= R, np.exp(-(r / s) ** 2 / 2), 0)
        approx = O.scale_filter_at(p, s)
        assert np.max(np.abs(approx - exact)) < 0.05


# ---------------------------------------------------------------- gradients

@pytest.fixture(scope="module")
def grad_case():
    H = blurred_noise((14, 13), 40).astype(np.float64)
    th = theta_field((14, 13), 41).astype(np.float64)
    comps, _ = O.angular_components(random_filter(7, 42, 2.0), 3)
    half = O.half_components(comps)
    g = np.random.default_rng(43).standard_normal(H.shape)
    return H, th, half, g


def _fd(f, x, idx, h=1e-6):
    xp = x.copy()
    xm = x.copy()
    xp[idx] += h
    xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


@pytest.mark.parametrize("op", ["conv", "corr"])
def test_gradients_match_finite_differences(grad_case, op):
    H, th, half, g = grad_case
    fwd = O.ext_conv_half if op == "conv" else O.ext_corr_half
    bwd = O.conv_backward if op == "conv" else O.corr_backward
    gH, gT, gF = bwd(H, th, half, g, route="direct")
    loss = lambda H_, th_, F_: np.sum(fwd(H_, th_, F_) * g)
    rng = np.random.default_rng(0)
    for _ in range(8):
        i, j = rng.integers(0, H.shape[0]), rng.integers(0, H.shape[1])
        assert gH[i, j] == pytest.approx(_fd(lambda x: loss(x, th, half), H, (i, j)), rel=1e-6, abs=1e-8)
        assert gT[i, j] == pytest.approx(_fd(lambda x: loss(H, x, half), th, (i, j)), rel=1e-6, abs=1e-8)
    for _ in range(8):
        k = rng.integers(0, half.shape[0])
        a, b = rng.integers(0, half.shape[1], 2)
        idx = (k, a, b)
        d_re = (loss(H, th, _bump(half, idx, 1e-6)) - loss(H, th, _bump(half, idx, -1e-6))) / 2e-6
        d_im = (loss(H, th, _bump(half, idx, 1e-6j)) - loss(H, th, _bump(half, idx, -1e-6j))) / 2e-6
        assert gF[idx].real == pytest.approx(d_re, rel=1e-6, abs=1e-8)
        assert gF[idx].imag == pytest.approx(d_im, rel=1e-6, abs=1e-8)


def _bump(a, idx, d):
    b = a.copy()
    b[idx] += d
    return b


@pytest.mark.parametrize("op", ["conv", "corr"])
def test_gradient_routes_agree(grad_case, op):
    H, th, half, g = grad_case
    bwd = O.conv_backward if op == "conv" else O.corr_backward
    a = bwd(H, th, half, g, route="direct")
    b = bwd(H, th, half, g, route="fft")
    for x, y in zip(a, b):
        assert rel(x, y) < 1e-12


def test_signal_gradient_dot_product(grad_case):
    """Linearity in H: <dL/dH, H> = L for both operators."""
    H, th, half, g = grad_case
    gH, _, _ = O.conv_backward(H, th, half, g)
    assert np.sum(gH * H) == pytest.approx(np.sum(O.ext_conv_half(H, th, half) * g), rel=1e-12)
    gH, _, _ = O.corr_backward(H, th, half, g)
    assert np.sum(gH * H) == pytest.approx(np.sum(O.ext_corr_half(H, th, half) * g), rel=1e-12)
