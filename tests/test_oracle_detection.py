"""Pins of the oracle's pattern detection (Sec. 5: gradient signal and field, consensus
filter by voting, peaks). CPU only."""
import numpy as np
import pytest
import scipy.ndimage as nd

import oracle as O
from synthetic import blurred_noise, matching_scene


def test_gradient_of_planes_and_axes():
    """A plane a x + b y has gradient (a, b) everywhere, one-sided differences included;
    its angle is atan2(b, a) with x along columns and y along rows."""
    yy, xx = np.mgrid[0:9, 0:11].astype(np.float64)
    for a, b in ((1.5, 0.0), (0.0, 2.0), (-1.0, 1.0), (0.3, -0.7)):
        H, th = O.gradient_field(a * xx + b * yy)
        assert np.allclose(H, np.hypot(a, b), atol=1e-13)
        assert np.allclose(np.cos(th), a / np.hypot(a, b), atol=1e-13)
        assert np.allclose(np.sin(th), b / np.hypot(a, b), atol=1e-13)


def test_single_edge_pixel_votes_once():
    """A pattern whose only non-zero gradient is at one pixel: the filter is that pixel's
    gradient magnitude split bilinearly around R_{-theta} (c - x)."""
    S, R = 11, 5
    P = np.zeros((S, S))
    P[2, 7] = 1.0                       # gradient non-zero at its four neighbours
    H, th = O.gradient_field(P)
    F = O.voting_filter(P)
    ref = np.zeros((S, S))
    for i, j in zip(*np.nonzero(H)):
        qx, qy = j - R, i - R
        if qx * qx + qy * qy > R * R:
            continue
        c, s = np.cos(th[i, j]), np.sin(th[i, j])
        px, py = c * -qx + s * -qy, -s * -qx + c * -qy
        # these four neighbours have axis-aligned gradients: integer vote positions
        assert abs(px - round(px)) < 1e-12 and abs(py - round(py)) < 1e-12
        ref[int(round(py)) + R, int(round(px)) + R] += H[i, j]
    assert np.allclose(F, ref, atol=1e-12)


def test_vote_mass_is_the_gradient_mass():
    """Bilinear splats keep each vote's weight: the filter sums to the gradient magnitude of
    the disk (all votes fall inside the window, since |c - x| <= R)."""
    P = blurred_noise((21, 21), 5).astype(np.float64)
    R = 10
    H, _ = O.gradient_field(P)
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    disk = xx * xx + yy * yy <= R * R
    # a vote at distance R may straddle the window edge by less than a pixel; the disk of
    # radius R - 1 votes entirely inside
    inner = xx * xx + yy * yy <= (R - 1) ** 2
    F = O.voting_filter(P)
    assert F.sum() <= H[disk].sum() + 1e-9
    assert F.sum() >= H[inner].sum() - 1e-9


def test_filter_is_invariant_to_quarter_turns_of_the_pattern():
    """Votes are expressed in the gradient's own frame, so turning the pattern by 90 degrees
    on the grid leaves the filter unchanged (up to rounding)."""
    _, pat, _ = matching_scene(256, 31, seeds=(1, 2, 3, 4))
    F = O.voting_filter(pat)
    for k in (1, 2, 3):
        assert np.max(np.abs(O.voting_filter(np.rot90(pat, k)) - F)) < 1e-10 * np.max(np.abs(F))


def test_peaks_are_the_maximum_filter_definition():
    """Peaks = pixels equal to the maximum of their (2r+1)^2 window and >= threshold
    (scipy.ndimage.maximum_filter), on data without ties."""
    D = np.random.default_rng(9).random((40, 53))
    r, thr = 3, 0.6
    mx = nd.maximum_filter(D, size=2 * r + 1, mode="constant", cval=-np.inf)
    ys, xs = np.nonzero((D == mx) & (D >= thr))
    rows, cols, vals = O.find_peaks(D, r, thr, 10 ** 6)
    assert sorted(zip(rows.tolist(), cols.tolist())) == sorted(zip(ys.tolist(), xs.tolist()))
    assert np.all(np.diff(vals) <= 0)


def test_peak_ties_go_to_the_first_pixel():
    D = np.zeros((5, 6))
    D[2, 1] = D[2, 3] = 1.0
    rows, cols, _ = O.find_peaks(D, 2, 0.5, 10)
    assert list(zip(rows, cols)) == [(2, 1)]


def test_detects_planted_patterns():
    """The scene of the matching workload at a reduced size: the three strongest peaks are
    the centres where the rotated pattern was pasted (Sec. 5: votes pile up at centres)."""
    img, pat, truth = matching_scene(384, 31, seeds=(30, 31, 32, 33))
    D, _ = O.detection_response(img, pat, 12)
    rows, cols, _ = O.find_peaks(D, 8, 0.3 * D.max(), 3)
    assert sorted(zip(rows.tolist(), cols.tolist())) == sorted((r, c) for r, c, _ in truth)
