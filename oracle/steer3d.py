"""Steering in 3D (Sec. 9): extended correlation and convolution of a volume with a filter
rotated by a per-voxel rotation, through spherical-harmonic components and Wigner-D
matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method (Sec. 9): write the filter as a sum over angular frequencies l <= K of
f_l^m(r) Y_l^m(direction), with f_l^m from a spherical-harmonic transform of F on every
radius; correlate the signal with the functions f_l^m(r) Y_l^{m'}(direction); combine
the results at every voxel with the Wigner-D coefficients of that voxel's rotation.

Readings (the paper states the idea; these make it a computation):

  V1  rotation action: (R F)(x) = F(R^{-1} x); the field gives R at every voxel as ZYZ
      Euler angles (alpha, beta, gamma), R = Rz(alpha) Ry(beta) Rz(gamma) (active,
      right-handed, acting on column vectors (x, y, z));
  V2  coordinates: a volume is indexed [z, y, x]; the filter's S x S x S array has its
      centre at (R, R, R), R = (S - 1) / 2, and voxel offset q = (x, y, z) = (column,
      row, slice) offsets; polar angle theta from +z, azimuth phi = atan2(y, x);
  V3  decomposition: the filter is restricted to the ball |x| <= R (closed under
      rotation); f_l^m(r) = integral over the unit sphere of F(r w) conj(Y_l^m(w)),
      evaluated at every distinct grid radius 0 < r <= R by quadrature: Gauss-Legendre
      in cos(theta) with M / 2 nodes times M equispaced azimuths, M the smallest power
      of two >= max(8 (2K + 1), 4 ceil(2 pi R)) (the 2D rule); F(r w) by trilinear
      interpolation of the array (zero outside it); the centre voxel keeps F(0) (l = 0);
  V4  spherical harmonics: orthonormal, Condon-Shortley phase (scipy's sph_harm_y);
  V5  Wigner-D: Y_l^m(R^{-1} x) = sum_{m'} D^l_{m'm}(R) Y_l^{m'}(x), so
      D^l_{m'm}(R) = integral of conj(Y_l^{m'}(w)) Y_l^m(R^{-1} w); for Euler angles
      D^l_{m'm} = e^{-i m' alpha} d^l_{m'm}(beta) e^{-i m gamma} with Wigner's explicit
      sum for d (the paper's formula conjugates D and swaps the roles of m and m', the
      same combination under the other convention for D);
  V6  components C_{l,m',m}(q) = f_l^m(|q|) Y_l^{m'}(q / |q|) on the ball (the centre:
      C_{0,0,0}(0) = F(0)); then (R F)(q) = sum D^l_{m'm}(R) C_{l,m',m}(q);
  V7  correlation y(p) = sum_q H(p + q) (R_p F)(q) = sum D^l_{m'm}(R_p) G_{l,m',m}(p),
      G = H correlated with C; convolution y(p) = sum_q H(q) (R_q F)(p - q) =
      sum ((H D^l_{m'm}(R_.)) convolved with C_{l,m',m})(p); zero outside the volume;
  V8  real filters: f_l^{-m} = (-1)^m conj f_l^m and the terms (m', m) and (-m', -m) are
      complex conjugates, so y = sum over the half set of w Re(D G): per l, m' = 0 with
      m = 0..l, then m' = 1..l with m = -l..l; w = 1 for the self-conjugate terms
      (l, 0, 0) and 2 for every other.

Pins (tests/test_oracle_steer3d.py): the explicit Wigner-D against its quadrature
definition, unitarity and the group law; the coefficients of filters whose trilinear
interpolation is exact and whose harmonic content is known in closed form (constants,
x, y, z, xy, xyz); the whole correlation and convolution against closed forms for
filters linear and bilinear in the coordinates under arbitrary rotation fields; brute
force (the rotated band-limited filter evaluated directly, no Wigner-D) = the FFT route.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y


def default_sphere_samples(K: int, R: int) -> int:
    """M (azimuths); the polar Gauss-Legendre rule has M / 2 nodes (V3)."""
    need = max(8 * (2 * K + 1), 4 * int(np.ceil(2.0 * np.pi * R)))
    M = 1
    while M < need:
        M *= 2
    return M


def trilinear(F, x, y, z):
    """Trilinear interpolation of the S^3 array F[z, y, x] at continuous offsets from its
    centre; samples outside the array count zero."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    R = (S - 1) // 2
    cs = [np.asarray(v, dtype=np.float64) + R for v in (x, y, z)]
    c0 = [np.floor(c).astype(np.int64) for c in cs]
    fr = [c - f for c, f in zip(cs, c0)]
    out = np.zeros(np.broadcast(*cs).shape, dtype=np.float64)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                ix, iy, iz = c0[0] + dx, c0[1] + dy, c0[2] + dz
                w = ((fr[0] if dx else 1.0 - fr[0]) * (fr[1] if dy else 1.0 - fr[1]) *
                     (fr[2] if dz else 1.0 - fr[2]))
                ok = (ix >= 0) & (ix < S) & (iy >= 0) & (iy < S) & (iz >= 0) & (iz < S)
                v = np.where(ok, F[np.clip(iz, 0, S - 1), np.clip(iy, 0, S - 1), np.clip(ix, 0, S - 1)], 0.0)
                out += w * v
    return out


def grid_radii3(R: int):
    """Distinct squared radii 0 < x^2 + y^2 + z^2 <= R^2 of the grid (sorted)."""
    d = np.arange(-R, R + 1)
    d2 = (d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2).ravel()
    return np.unique(d2[(d2 > 0) & (d2 <= R * R)])


def sh_coefficients(F, K: int, M: int = 0):
    """(d2list, f) with f[i, l, m + K] = f_l^m(sqrt(d2list[i])) for l <= K, |m| <= l (V3);
    entries with |m| > l are zero."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    R = (S - 1) // 2
    M = M or default_sphere_samples(K, R)
    nt = M // 2
    t, wt = np.polynomial.legendre.leggauss(nt)
    theta = np.arccos(t)
    phi = 2.0 * np.pi * np.arange(M) / M
    d2list = grid_radii3(R)
    r = np.sqrt(d2list.astype(np.float64))
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    ux, uy, uz = st * np.cos(phi)[None, :], st * np.sin(phi)[None, :], np.broadcast_to(ct, (nt, M))
    samples = trilinear(F, r[:, None, None] * ux, r[:, None, None] * uy, r[:, None, None] * uz)   # [nr, nt, M]
    f = np.zeros((len(r), K + 1, 2 * K + 1), dtype=np.complex128)
    quad = (wt[:, None] * (2.0 * np.pi / M))
    for l in range(K + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, m, theta[:, None], phi[None, :])                  # [nt, M]
            f[:, l, m + K] = np.einsum("rij,ij->r", samples, np.conj(Y) * quad)
    return d2list, f


def half_set(K: int):
    """(l, m', m, weight) of the half set in order (V8)."""
    out = []
    for l in range(K + 1):
        for m in range(0, l + 1):
            out.append((l, 0, m, 1.0 if m == 0 else 2.0))
        for mp in range(1, l + 1):
            for m in range(-l, l + 1):
                out.append((l, mp, m, 2.0))
    return out


def _voxel_directions(R: int):
    d = np.arange(-R, R + 1, dtype=np.float64)
    z, y, x = np.meshgrid(d, d, d, indexing="ij")
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    theta = np.arccos(np.where(r > 0, z / np.where(r > 0, r, 1.0), 1.0))
    phi = np.arctan2(y, x)
    return x, y, z, r2.astype(np.int64), theta, phi


def components3d(F, K: int, M: int = 0):
    """(hs, comps) with hs = half_set(K) and comps[c] the S^3 complex component of hs[c]
    (V6)."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    R = (S - 1) // 2
    d2list, f = sh_coefficients(F, K, M)
    idx = {int(v): i for i, v in enumerate(d2list)}
    x, y, z, r2, theta, phi = _voxel_directions(R)
    inside = (r2 > 0) & (r2 <= R * R)
    ri = np.vectorize(lambda v: idx.get(int(v), 0))(r2)
    hs = half_set(K)
    comps = np.zeros((len(hs), S, S, S), dtype=np.complex128)
    for c, (l, mp, m, _) in enumerate(hs):
        val = f[ri, l, m + K] * sph_harm_y(l, mp, theta, phi)
        comps[c] = np.where(inside, val, 0.0)
        if l == 0:
            comps[c][R, R, R] = F[R, R, R]
    return hs, comps


def euler_matrix(alpha, beta, gamma):
    """R = Rz(alpha) Ry(beta) Rz(gamma), shape (..., 3, 3) (V1)."""
    a, b, g = (np.asarray(v, dtype=np.float64) for v in (alpha, beta, gamma))

    def rz(t):
        c, s = np.cos(t), np.sin(t)
        o, i = np.zeros_like(t), np.ones_like(t)
        return np.stack([np.stack([c, -s, o], -1), np.stack([s, c, o], -1), np.stack([o, o, i], -1)], -2)

    def ry(t):
        c, s = np.cos(t), np.sin(t)
        o, i = np.zeros_like(t), np.ones_like(t)
        return np.stack([np.stack([c, o, s], -1), np.stack([o, i, o], -1), np.stack([-s, o, c], -1)], -2)

    return rz(a) @ ry(b) @ rz(g)


def wigner_small_d(l: int, beta):
    """d^l_{m'm}(beta), shape (..., 2l + 1, 2l + 1) indexed [m' + l, m + l]: Wigner's
    explicit sum (V5)."""
    beta = np.asarray(beta, dtype=np.float64)
    c, s = np.cos(beta / 2.0), np.sin(beta / 2.0)
    out = np.zeros(beta.shape + (2 * l + 1, 2 * l + 1), dtype=np.float64)
    fac = math.factorial
    for mp in range(-l, l + 1):
        for m in range(-l, l + 1):
            pre = math.sqrt(fac(l + mp) * fac(l - mp) * fac(l + m) * fac(l - m))
            acc = np.zeros_like(beta)
            for k in range(max(0, m - mp), min(l + m, l - mp) + 1):
                coef = (-1.0) ** (mp - m + k) * pre / (fac(l + m - k) * fac(k) * fac(mp - m + k) * fac(l - mp - k))
                acc = acc + coef * c ** (2 * l + m - mp - 2 * k) * s ** (mp - m + 2 * k)
            out[..., mp + l, m + l] = acc
    return out


def wigner_D(l: int, alpha, beta, gamma):
    """D^l_{m'm}(alpha, beta, gamma) = e^{-i m' alpha} d^l_{m'm}(beta) e^{-i m gamma} (V5)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    ms = np.arange(-l, l + 1)
    ea = np.exp(-1j * alpha[..., None] * ms)        # [..., m']
    eg = np.exp(-1j * gamma[..., None] * ms)        # [..., m]
    return ea[..., :, None] * wigner_small_d(l, beta) * eg[..., None, :]


def wigner_D_quadrature(l: int, Rmat):
    """The definition (V5) by quadrature, exact for degree-l harmonics: D^l_{m'm}(R) =
    integral conj(Y_l^{m'}(w)) Y_l^m(R^{-1} w)."""
    nt, M = l + 2, 2 * l + 4
    t, wt = np.polynomial.legendre.leggauss(nt)
    theta = np.arccos(t)[:, None] * np.ones((1, M))
    phi = (2.0 * np.pi * np.arange(M) / M)[None, :] * np.ones((nt, 1))
    w = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)
    v = w @ np.asarray(Rmat, dtype=np.float64)          # rows: R^T w = R^{-1} w
    th2 = np.arccos(np.clip(v[..., 2], -1.0, 1.0))
    ph2 = np.arctan2(v[..., 1], v[..., 0])
    quad = wt[:, None] * (2.0 * np.pi / M)
    D = np.zeros((2 * l + 1, 2 * l + 1), dtype=np.complex128)
    for mp in range(-l, l + 1):
        Yp = np.conj(sph_harm_y(l, mp, theta, phi))
        for m in range(-l, l + 1):
            D[mp + l, m + l] = np.sum(quad * Yp * sph_harm_y(l, m, th2, ph2))
    return D


def rotated_band_limited(F, K: int, Rmat, M: int = 0, coeffs=None):
    """(R F~)(q) on the S^3 grid for one rotation, F~ the band-limited filter: the sum over
    all l <= K, |m| <= l of f_l^m(|q|) Y_l^m(R^{-1} q / |q|), evaluated directly (real
    part; the centre keeps F(0)). coeffs: sh_coefficients(F, K, M) if already known."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    R = (S - 1) // 2
    d2list, f = coeffs if coeffs is not None else sh_coefficients(F, K, M)
    idx = {int(v): i for i, v in enumerate(d2list)}
    x, y, z, r2, _, _ = _voxel_directions(R)
    inside = (r2 > 0) & (r2 <= R * R)
    ri = np.vectorize(lambda v: idx.get(int(v), 0))(r2)
    q = np.stack([x, y, z], -1)
    v = q @ np.asarray(Rmat, dtype=np.float64)          # R^{-1} q (rows times R = R^T q)
    rr = np.sqrt(np.sum(v * v, -1))
    th = np.arccos(np.clip(np.where(rr > 0, v[..., 2] / np.where(rr > 0, rr, 1.0), 1.0), -1.0, 1.0))
    ph = np.arctan2(v[..., 1], v[..., 0])
    acc = np.zeros((S, S, S), dtype=np.complex128)
    for l in range(K + 1):
        for m in range(-l, l + 1):
            acc += f[ri, l, m + K] * sph_harm_y(l, m, th, ph)
    out = np.where(inside, acc.real, 0.0)
    out[R, R, R] = F[R, R, R]
    return out


def ext_corr3d_brute(H, alpha, beta, gamma, F, K: int, M: int = 0):
    """Extended correlation by the definition (V7): y(p) = sum_q H(p + q) (R_p F~)(q), the
    rotated filter evaluated per voxel without Wigner-D. Small volumes only."""
    H = np.asarray(H, dtype=np.float64)
    S = np.asarray(F).shape[0]
    R = (S - 1) // 2
    nz, ny, nx = H.shape
    Rm = euler_matrix(alpha, beta, gamma)
    co = sh_coefficients(F, K, M)
    Hp = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
    Hp[R:R + nz, R:R + ny, R:R + nx] = H
    y = np.zeros((nz, ny, nx))
    for k in range(nz):
        for i in range(ny):
            for j in range(nx):
                filt = rotated_band_limited(F, K, Rm[k, i, j], M, co)
                y[k, i, j] = np.sum(Hp[k:k + S, i:i + S, j:j + S] * filt)
    return y


def ext_conv3d_brute(H, alpha, beta, gamma, F, K: int, M: int = 0):
    """Extended convolution by the definition (V7): every voxel q scatters H(q) times its
    rotated filter, y(p) = sum_q H(q) (R_q F~)(p - q). Small volumes only."""
    H = np.asarray(H, dtype=np.float64)
    S = np.asarray(F).shape[0]
    R = (S - 1) // 2
    nz, ny, nx = H.shape
    Rm = euler_matrix(alpha, beta, gamma)
    co = sh_coefficients(F, K, M)
    yp = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
    for k in range(nz):
        for i in range(ny):
            for j in range(nx):
                if H[k, i, j] == 0.0:
                    continue
                # p = q + x for the filter offset x: array entry a of the window is x = a - R
                filt = rotated_band_limited(F, K, Rm[k, i, j], M, co)
                yp[k:k + S, i:i + S, j:j + S] += H[k, i, j] * filt
    return yp[R:R + nz, R:R + ny, R:R + nx]


def _D_half(hs, alpha, beta, gamma):
    """D^l_{m'm} at every voxel for every half-set entry: [U, nz, ny, nx] complex."""
    Ds = {}
    out = []
    for (l, mp, m, _) in hs:
        if l not in Ds:
            Ds[l] = wigner_D(l, alpha, beta, gamma)
        out.append(Ds[l][..., mp + l, m + l])
    return np.array(out)


def fft_size3(n: int, R: int) -> int:
    return n + R


def ext_corr3d_fft(H, alpha, beta, gamma, F, K: int, M: int = 0, parts=None):
    """The FFT route of Sec. 9 (V7, V8): G_c = H correlated with C_c by zero-padded 3D FFTs
    of n + R per axis, y = sum_c w_c Re(D_c G_c). parts: components3d(F, K, M) if known."""
    H = np.asarray(H, dtype=np.float64)
    S = np.asarray(F).shape[0]
    R = (S - 1) // 2
    nz, ny, nx = H.shape
    P = (nz + R, ny + R, nx + R)
    hs, comps = parts if parts is not None else components3d(F, K, M)
    D = _D_half(hs, alpha, beta, gamma)
    Hf = np.fft.fftn(H, s=P, axes=(0, 1, 2))
    idx = np.arange(-R, R + 1)
    y = np.zeros((nz, ny, nx))
    for c, (l, mp, m, w) in enumerate(hs):
        # correlation = convolution with C(-q): place C(q) at (-q) mod P
        placed = np.zeros(P, dtype=np.complex128)
        placed[np.ix_((-idx) % P[0], (-idx) % P[1], (-idx) % P[2])] = comps[c]
        G = np.fft.ifftn(Hf * np.fft.fftn(placed))[:nz, :ny, :nx]
        y += w * np.real(D[c] * G)
    return y


def ext_conv3d_fft(H, alpha, beta, gamma, F, K: int, M: int = 0, parts=None):
    """Convolution by the FFT route (V7, V8): y = Re sum_c w_c ((H D_c) convolved with C_c).
    parts: components3d(F, K, M) if known."""
    H = np.asarray(H, dtype=np.float64)
    S = np.asarray(F).shape[0]
    R = (S - 1) // 2
    nz, ny, nx = H.shape
    P = (nz + R, ny + R, nx + R)
    hs, comps = parts if parts is not None else components3d(F, K, M)
    D = _D_half(hs, alpha, beta, gamma)
    idx = np.arange(-R, R + 1)
    acc = np.zeros(P, dtype=np.complex128)
    for c, (l, mp, m, w) in enumerate(hs):
        placed = np.zeros(P, dtype=np.complex128)
        placed[np.ix_(idx % P[0], idx % P[1], idx % P[2])] = comps[c]
        acc += w * np.fft.fftn(H * D[c], s=P, axes=(0, 1, 2)) * np.fft.fftn(placed)
    return np.real(np.fft.ifftn(acc)[:nz, :ny, :nx])
