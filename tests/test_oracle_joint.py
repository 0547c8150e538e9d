"""Pins of the oracle's joint rotation and scale fields (product of the rotation and scale
decompositions). CPU only. The coefficients c_{k,l} themselves are parity-unpinned (they
follow only from the readings); what is pinned is what must hold for any coefficients."""
import numpy as np
import pytest
import scipy.signal as ss

import oracle as O
from oracle.joint import JointParams, joint_components, joint_conv_brute, joint_conv_fft, joint_filter_at, joint_smooth
from synthetic import anisotropic_gaussian, blurred_noise, scale_field, theta_field

P = JointParams(K=4, n_log=7, s_min=1.0, s_max=2.0, period_factor=1.5)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def case():
    H = blurred_noise((19, 23), 40).astype(np.float64)
    th = theta_field((19, 23), 41).astype(np.float64)
    s = scale_field((19, 23), 42, 1.0, 2.0, sigma=3.0).astype(np.float64)
    F = anisotropic_gaussian(9, 2.5, 1.0).astype(np.float64)
    return H, th, s, F


def test_brute_force_equals_fft_route(case):
    H, th, s, F = case
    assert rel(joint_conv_fft(H, th, s, F, P), joint_conv_brute(H, th, s, F, P)) < 1e-12
    assert rel(joint_conv_fft(H, th, s, F, P, True), joint_conv_brute(H, th, s, F, P, True)) < 1e-12


def test_constant_fields_are_a_textbook_convolution(case):
    """Constant theta and s: the extended convolution is scipy's convolution with the
    transformed band-limited filter."""
    H, _, _, F = case
    for t0, s0 in ((0.0, 1.0), (0.8, 1.3), (2.9, 2.0)):
        Ft = joint_filter_at(F, P, t0, s0)
        y = joint_conv_brute(H, np.full(H.shape, t0), np.full(H.shape, s0), F, P)
        assert rel(y, ss.convolve2d(H, Ft, mode="same", boundary="fill")) < 1e-12


def test_real_half_set_and_centre(case):
    """The half set carries every pair (k, l), (-k, -l) once; the centre is fixed by every
    transformation."""
    _, _, _, F = case
    ks, ls, ws, comps = joint_components(F, P)
    h = (P.n_log - 1) // 2
    assert len(ks) == (P.K + 1) * P.n_log - h
    assert sorted(set(zip(ks.tolist(), ls.tolist()))) == sorted(zip(ks.tolist(), ls.tolist()))
    R = (F.shape[0] - 1) // 2
    for t0, s0 in ((0.3, 1.0), (1.7, 1.9)):
        assert joint_filter_at(F, P, t0, s0)[R, R] == pytest.approx(F[R, R], abs=1e-15)


def test_transformed_filter_follows_rotation_and_scale(case):
    """The transformed band-limited filter approximates F(R_{-theta} x / s): quarter turns
    are exact on the grid (same samples), other transformations close to the analytic
    anisotropic Gaussian."""
    _, _, _, F = case
    F0 = joint_filter_at(F, P, 0.0, 1.0)
    assert np.max(np.abs(joint_filter_at(F, P, np.pi / 2, 1.0) - np.rot90(F0, -1))) < 1e-12 * np.max(np.abs(F0))
    R = (F.shape[0] - 1) // 2
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    for t0, s0 in ((0.6, 1.4), (2.2, 1.8)):
        xr = (np.cos(t0) * xx + np.sin(t0) * yy) / s0     # R_{-theta} x / s
        yr = (-np.sin(t0) * xx + np.cos(t0) * yy) / s0
        ana = np.exp(-xr ** 2 / (2 * 2.5 ** 2) - yr ** 2 / (2 * 1.0 ** 2))
        disk = xx ** 2 + yy ** 2 <= R * R
        err = np.max(np.abs(joint_filter_at(F, P, t0, s0) - ana)[disk])
        assert err < 0.15, err     # band-limited (K = 4, 7 log-radial modes) approximation


def test_quarter_turn_equivariance(case):
    H, th, s, F = case
    Hs = H[:19, :19]
    ths, sss = th[:19, :19], s[:19, :19]
    a = joint_conv_brute(np.rot90(Hs), np.rot90(ths) - np.pi / 2, np.rot90(sss), F, P)
    b = joint_conv_brute(Hs, ths, sss, F, P)
    assert rel(a, np.rot90(b)) < 1e-12


def test_normalised_smoothing_preserves_constants(case):
    _, th, s, F = case
    y, _, den = joint_smooth(np.full(th.shape, 0.42), th, s, F, P, route="brute")
    assert np.min(den) > 0
    assert np.max(np.abs(y - 0.42)) < 1e-13
