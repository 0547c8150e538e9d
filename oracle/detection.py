"""Pattern detection by extended convolution (Sec. 5, Application to Pattern Detection).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the section's order:
  * signal and field (eq. signal, eq. theta): H = |grad I| and theta = atan2(dI/dy, dI/dx)
    of the target image;
  * the consensus filter (eq. opt_filt; appendix "Defining Optimal Filters"): every pixel x
    of the pattern within radius R of its centre c votes with weight |grad P(x)| for the
    position of c seen from the frame at x whose first axis is the gradient direction,
    i.e. at R_{-theta_P(x)} (c - x);
  * the extended convolution of {H, theta} with the band-limited decomposition of that
    filter (eq. Def-EConv, Sec. 4.1): every image pixel scatters its vote, so instances of
    the pattern at any rotation pile their votes up at their centres;
  * peak picking on the response.

Readings (the section leaves them open):
  * gradient: central differences inside, one-sided differences on the border rows and
    columns (numpy.gradient with unit spacing); x = column, y = row (as everywhere else);
  * a vote at a non-integer position is split over the four surrounding bins with bilinear
    weights; votes landing outside the S x S window are dropped; S = the pattern's side
    and R = (S - 1) / 2 (the disk of the decomposition);
  * the filter is rounded to float32 before its decomposition (the library's plans take
    float32 filters);
  * a peak is a pixel whose response is >= `threshold` and not below any response within
    the (2r+1) x (2r+1) window around it, ties going to the first pixel in raster order;
    peaks are listed by decreasing response (ties by raster index).
"""
from __future__ import annotations

import numpy as np

from .decompose import angular_components, half_components
from .extended import ext_conv_half


def gradient_field(I):
    """(H, theta) = (|grad I|, atan2(I_y, I_x)) by central differences (one-sided on the
    border)."""
    I = np.asarray(I, dtype=np.float64)
    gy, gx = np.gradient(I)          # axis 0 = rows (y), axis 1 = columns (x)
    return np.hypot(gx, gy), np.arctan2(gy, gx)


def voting_filter(P):
    """Consensus filter of an S x S pattern (S odd): the sum over pattern pixels x with
    |x - c| <= R of |grad P(x)| times a unit vote at R_{-theta_P(x)} (c - x), split
    bilinearly over the window's bins. Returns the S x S float64 filter (row = y, col = x,
    centre at (R, R))."""
    P = np.asarray(P, dtype=np.float64)
    S = P.shape[0]
    assert P.shape == (S, S) and S % 2 == 1
    R = (S - 1) // 2
    H, th = gradient_field(P)
    F = np.zeros((S, S))
    for i in range(S):
        for j in range(S):
            qx, qy = j - R, i - R          # x - c
            if qx * qx + qy * qy > R * R or H[i, j] == 0.0:
                continue
            c, s = np.cos(th[i, j]), np.sin(th[i, j])
            vx, vy = -qx, -qy              # c - x
            px = c * vx + s * vy           # R_{-theta} (c - x)
            py = -s * vx + c * vy
            fx, fy = px + R, py + R        # window coordinates (column, row)
            x0, y0 = int(np.floor(fx)), int(np.floor(fy))
            ax, ay = fx - x0, fy - y0
            for dy, wy in ((0, 1.0 - ay), (1, ay)):
                for dx, wx in ((0, 1.0 - ax), (1, ax)):
                    r_, c_ = y0 + dy, x0 + dx
                    if 0 <= r_ < S and 0 <= c_ < S:
                        F[r_, c_] += H[i, j] * wy * wx
    return F


def find_peaks(D, radius, threshold, max_peaks):
    """Local maxima of D (see the module's reading), at most max_peaks of them, as
    (rows, cols, values) sorted by decreasing value, ties by raster index."""
    D = np.asarray(D, dtype=np.float64)
    ny, nx = D.shape
    rows, cols, vals = [], [], []
    for y, x in np.argwhere(D >= threshold):     # candidates, in raster order
        y, x = int(y), int(x)
        v = D[y, x]
        ok = True
        for yy in range(max(0, y - radius), min(ny, y + radius + 1)):
            for xx in range(max(0, x - radius), min(nx, x + radius + 1)):
                w = D[yy, xx]
                earlier = yy * nx + xx < y * nx + x
                if w > v or (earlier and w == v):
                    ok = False
                    break
            if not ok:
                break
        if ok:
            rows.append(y)
            cols.append(x)
            vals.append(v)
    order = sorted(range(len(vals)), key=lambda k: (-vals[k], rows[k] * nx + cols[k]))[:max_peaks]
    return (np.array([rows[k] for k in order], dtype=np.int64), np.array([cols[k] for k in order], dtype=np.int64),
            np.array([vals[k] for k in order]))


def detection_response(I, P, K):
    """Votes for pattern centres: {|grad I|, atan2 grad I} * F (extended convolution with the
    band-limited decomposition of the float32-rounded consensus filter of P)."""
    H, th = gradient_field(I)
    F = voting_filter(P).astype(np.float32)
    comps, _ = angular_components(F, K)
    return ext_conv_half(H, th, half_components(comps)), F
