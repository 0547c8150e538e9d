"""Angular-frequency decomposition of a filter (Sec. 4.1, "Filter Decomposition").

The paper writes the filter in polar coordinates and runs a 1D FFT over angle at
each radius, giving F = sum_k F_k with F_k(r, phi) = f_k(r) e^{i k phi}.
Rotating F by an angle Theta multiplies F_k by e^{-i k Theta} (Sec. 3, example
n = 1; Sec. 4.1), i.e. (T_Theta F)(r, phi) = F(r, phi - Theta).

Readings (the paper is silent on these):
  * coordinates: x = (dx, dy) with dx = column offset (right), dy = row offset
    (down); phi(x) = atan2(dy, dx); array index F[R + dy, R + dx];
  * polar samples: bilinear interpolation of the S x S array (zero outside it),
    at the exact distinct grid radii rho = |x| (0 < rho <= R) and M equispaced
    angles phi_m = 2 pi m / M;
  * support: the disk |x| <= R, which is closed under rotation;
  * centre pixel: F_k(0) = F(0) for k = 0 and 0 otherwise;
  * band limit: hard truncation to k = -K..K (Sec. 4.3).
"""
from __future__ import annotations

import numpy as np


def default_angular_samples(K: int, R: int) -> int:
    """Number of angular samples M: the smallest power of two that is at least
    8 (2K+1) and at least 4 ceil(2 pi R) (enough to resolve the outer ring)."""
    need = max(8 * (2 * K + 1), 4 * int(np.ceil(2.0 * np.pi * R)))
    M = 1
    while M < need:
        M *= 2
    return M


def bilinear(F: np.ndarray, dx, dy):
    """Bilinear interpolation of the S x S array F at continuous offsets (dx, dy)
    from its centre. Samples outside the array contribute zero."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    R = (S - 1) // 2
    col = np.asarray(dx, dtype=np.float64) + R
    row = np.asarray(dy, dtype=np.float64) + R
    c0 = np.floor(col).astype(np.int64)
    r0 = np.floor(row).astype(np.int64)
    fc = col - c0
    fr = row - r0
    out = np.zeros(np.broadcast(col, row).shape, dtype=np.float64)
    for rr, wr in ((r0, 1.0 - fr), (r0 + 1, fr)):
        for cc, wc in ((c0, 1.0 - fc), (c0 + 1, fc)):
            ok = (rr >= 0) & (rr < S) & (cc >= 0) & (cc < S)
            val = np.where(ok, F[np.clip(rr, 0, S - 1), np.clip(cc, 0, S - 1)], 0.0)
            out += wr * wc * val
    return out


def grid_radii(R: int):
    """Distinct squared radii d2 = dx^2 + dy^2 with 0 < d2 <= R^2 (sorted)."""
    d = np.arange(-R, R + 1)
    d2 = (d[:, None] ** 2 + d[None, :] ** 2).ravel()
    return np.unique(d2[(d2 > 0) & (d2 <= R * R)])


def angular_components(F, K: int, M: int | None = None):
    """Components F_k, k = -K..K, of the S x S filter F on the grid.

    Returns (comps, f) where comps has shape (2K+1, S, S), complex128, index k+K,
    and f maps each distinct squared radius to the vector f_k(rho), k = -K..K.
    f_k(rho) = (1/M) sum_m F(rho cos phi_m, rho sin phi_m) e^{-i k phi_m}
    (the per-radius angular DFT of Sec. 4.1), and
    F_k(x) = f_k(|x|) e^{i k phi(x)} on the disk.
    """
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    assert F.shape == (S, S) and S % 2 == 1
    R = (S - 1) // 2
    if M is None:
        M = default_angular_samples(K, R)
    assert 0 <= K <= M // 2 - 1
    ks = np.arange(-K, K + 1)
    phis = 2.0 * np.pi * np.arange(M) / M
    f = {}
    for d2 in grid_radii(R):
        rho = np.sqrt(float(d2))
        v = bilinear(F, rho * np.cos(phis), rho * np.sin(phis))        # v_m
        f[int(d2)] = (np.exp(-1j * np.outer(ks, phis)) @ v) / M           # f_k(rho)
    comps = np.zeros((2 * K + 1, S, S), dtype=np.complex128)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            d2 = dx * dx + dy * dy
            if d2 == 0 or d2 > R * R:
                continue
            phi = np.arctan2(dy, dx)
            comps[:, R + dy, R + dx] = f[d2] * np.exp(1j * ks * phi)
    comps[K, R, R] = F[R, R]
    return comps, f


def rotated_filter(comps, theta: float):
    """The band-limited filter rotated by theta: F_theta = sum_k e^{-i k theta} F_k
    (rotation multiplies the k-th angular component by e^{-i k theta}, Sec. 4.1)."""
    comps = np.asarray(comps)
    K = (comps.shape[0] - 1) // 2
    ks = np.arange(-K, K + 1)
    return np.tensordot(np.exp(-1j * ks * theta), comps, axes=1)


def half_components(comps):
    """The k = 0..K half of a full component stack (k = -K..K)."""
    K = (comps.shape[0] - 1) // 2
    return np.asarray(comps)[K:]
