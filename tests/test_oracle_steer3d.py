"""Pins of the 3D steering oracle (Sec. 9) against what the mathematics fixes.

* Wigner-D: Wigner's explicit sum against its definition as the matrix of a rotation in
  the spherical-harmonic basis (quadrature with scipy's harmonics), unitarity, group law.
* Spherical-harmonic coefficients of filters whose trilinear interpolation is exact and
  whose harmonic content is textbook: a constant (l = 0), x, y, z (l = 1), xy (l = 2),
  xyz (l = 3), with the orthonormal harmonics' constants written out here.
* Whole correlation / convolution under random rotation fields against closed forms: a
  filter a . q (rotated: (R a) . q) and the filter q_x q_y (rotated: (R^T q)_x (R^T q)_y).
* Brute force (rotated band-limited filter synthesised per voxel, no Wigner-D) = the FFT
  route with Wigner-D, for a random filter.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import steer3d as O3


def rot_field(shape, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-np.pi, np.pi, shape)
    b = np.arccos(rng.uniform(-1.0, 1.0, shape))
    g = rng.uniform(-np.pi, np.pi, shape)
    return a, b, g


def grid(S):
    R = (S - 1) // 2
    d = np.arange(-R, R + 1, dtype=np.float64)
    z, y, x = np.meshgrid(d, d, d, indexing="ij")
    return x, y, z


@pytest.mark.parametrize("l", range(6))
def test_wigner_d_matches_its_definition(l):
    rng = np.random.default_rng(100 + l)
    for _ in range(4):
        a, b, g = rng.uniform(-np.pi, np.pi, 3)
        D = O3.wigner_D(l, a, b, g)
        Dq = O3.wigner_D_quadrature(l, O3.euler_matrix(a, b, g))
        assert np.max(np.abs(D - Dq)) <= 1e-12


def test_wigner_D_unitary_and_group_law():
    rng = np.random.default_rng(7)
    for l in (1, 2, 4):
        e1, e2 = rng.uniform(-np.pi, np.pi, 3), rng.uniform(-np.pi, np.pi, 3)
        D1, D2 = O3.wigner_D(l, *e1), O3.wigner_D(l, *e2)
        assert np.allclose(D1 @ D1.conj().T, np.eye(2 * l + 1), atol=1e-12)
        R12 = O3.euler_matrix(*e1) @ O3.euler_matrix(*e2)
        assert np.max(np.abs(O3.wigner_D_quadrature(l, R12) - D1 @ D2)) <= 1e-12
    # a rotation about z by a: D = diag(e^{-i m a})
    a = 0.7
    assert np.allclose(O3.wigner_D(3, a, 0.0, 0.0), np.diag(np.exp(-1j * a * np.arange(-3, 4))), atol=1e-14)


def test_trilinear_matches_scipy_map_coordinates():
    rng = np.random.default_rng(3)
    F = rng.standard_normal((7, 7, 7))
    pts = rng.uniform(-3.5, 3.5, (3, 200))
    got = O3.trilinear(F, pts[0], pts[1], pts[2])
    ref = ndimage.map_coordinates(F, [pts[2] + 3, pts[1] + 3, pts[0] + 3], order=1, mode="grid-constant", cval=0.0)
    assert np.max(np.abs(got - ref)) <= 1e-12


def coeff_expectations(name, r, K):
    """f[l, m + K] of the named filter at radius r from the orthonormal harmonics:
    Y_1^{+-1} = -+ sqrt(3 / 8 pi) sin t e^{+-i p}, Y_1^0 = sqrt(3 / 4 pi) cos t,
    Y_2^{+-2} = (1/4) sqrt(15 / 2 pi) sin^2 t e^{+-2ip},
    Y_3^{+-2} = (1/4) sqrt(105 / 2 pi) sin^2 t cos t e^{+-2ip}."""
    e = np.zeros((K + 1, 2 * K + 1), dtype=np.complex128)
    s1 = np.sqrt(2 * np.pi / 3)
    if name == "const":
        e[0, K] = 2.5 * np.sqrt(4 * np.pi)
    elif name == "x":
        e[1, K + 1], e[1, K - 1] = -r * s1, r * s1
    elif name == "y":
        e[1, K + 1], e[1, K - 1] = 1j * r * s1, 1j * r * s1
    elif name == "z":
        e[1, K] = r * np.sqrt(4 * np.pi / 3)
    elif name == "xy":
        c2 = 0.25 * np.sqrt(15 / (2 * np.pi))
        e[2, K + 2], e[2, K - 2] = -1j * r ** 2 / (4 * c2), 1j * r ** 2 / (4 * c2)
    elif name == "xyz":
        c3 = 0.25 * np.sqrt(105 / (2 * np.pi))
        e[3, K + 2], e[3, K - 2] = -1j * r ** 3 / (4 * c3), 1j * r ** 3 / (4 * c3)
    return e


@pytest.mark.parametrize("name", ["const", "x", "y", "z", "xy", "xyz"])
def test_sh_coefficients_closed_forms(name):
    S, K = 7, 4
    x, y, z = grid(S)
    F = {"const": np.full_like(x, 2.5), "x": x, "y": y, "z": z, "xy": x * y, "xyz": x * y * z}[name]
    d2list, f = O3.sh_coefficients(F, K)
    assert len(d2list) > 5
    for i, d2 in enumerate(d2list):
        e = coeff_expectations(name, np.sqrt(d2), K)
        assert np.max(np.abs(f[i] - e)) <= 1e-11 * max(1.0, float(d2) ** 1.5), (name, d2)


def test_half_set_reconstructs_the_band_limited_filter():
    """At the identity rotation the half-set sum of w Re C over the terms m' = m equals the
    full sum over l, m of f_l^m Y_l^m, synthesised directly."""
    rng = np.random.default_rng(5)
    S, K = 7, 3
    F = rng.standard_normal((S, S, S))
    hs, comps = O3.components3d(F, K)
    assert len(hs) == sum(2 * l * l + 2 * l + 1 for l in range(K + 1))
    w = np.array([h[3] for h in hs])
    # identity rotation: D = I, so only the m' = m terms survive
    diag = np.array([1.0 if h[1] == h[2] else 0.0 for h in hs])
    rec_id = np.tensordot(w * diag, comps.real, axes=1)
    ref = O3.rotated_band_limited(F, K, np.eye(3))
    assert np.max(np.abs(rec_id - ref)) <= 1e-12 * np.max(np.abs(ref))


def closed_corr(H, Rm, fn, S):
    R = (S - 1) // 2
    nz, ny, nx = H.shape
    x, y, z = grid(S)
    ball = x * x + y * y + z * z <= R * R
    q = np.stack([x, y, z], -1)
    Hp = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
    Hp[R:R + nz, R:R + ny, R:R + nx] = H
    out = np.zeros_like(H, dtype=np.float64)
    for k in range(nz):
        for i in range(ny):
            for j in range(nx):
                v = q @ Rm[k, i, j]                  # R^{-1} q
                out[k, i, j] = np.sum(Hp[k:k + S, i:i + S, j:j + S] * np.where(ball, fn(v), 0.0))
    return out


def closed_conv(H, Rm, fn, S):
    R = (S - 1) // 2
    nz, ny, nx = H.shape
    x, y, z = grid(S)
    ball = x * x + y * y + z * z <= R * R
    q = np.stack([x, y, z], -1)
    yp = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
    for k in range(nz):
        for i in range(ny):
            for j in range(nx):
                v = q @ Rm[k, i, j]
                yp[k:k + S, i:i + S, j:j + S] += H[k, i, j] * np.where(ball, fn(v), 0.0)
    return yp[R:R + nz, R:R + ny, R:R + nx]


FILTERS = {
    "linear": (lambda v: v[..., 0] * 0.3 - v[..., 1] * 1.1 + v[..., 2] * 0.7, 1),
    "bilinear": (lambda v: v[..., 0] * v[..., 1], 2),
}


@pytest.mark.parametrize("fname", list(FILTERS))
@pytest.mark.parametrize("route", ["brute", "fft"])
def test_correlation_closed_form(fname, route):
    fn, lmin = FILTERS[fname]
    S = 7
    x, y, z = grid(S)
    F = fn(np.stack([x, y, z], -1))
    H = np.random.default_rng(11).standard_normal((4, 5, 6))
    a, b, g = rot_field(H.shape, 12)
    ref = closed_corr(H, O3.euler_matrix(a, b, g), fn, S)
    f = O3.ext_corr3d_brute if route == "brute" else O3.ext_corr3d_fft
    got = f(H, a, b, g, F, lmin + 1)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("fname", list(FILTERS))
@pytest.mark.parametrize("route", ["brute", "fft"])
def test_convolution_closed_form(fname, route):
    fn, lmin = FILTERS[fname]
    S = 7
    x, y, z = grid(S)
    F = fn(np.stack([x, y, z], -1))
    H = np.random.default_rng(13).standard_normal((5, 4, 6))
    a, b, g = rot_field(H.shape, 14)
    ref = closed_conv(H, O3.euler_matrix(a, b, g), fn, S)
    f = O3.ext_conv3d_brute if route == "brute" else O3.ext_conv3d_fft
    got = f(H, a, b, g, F, lmin)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_brute_force_equals_fft_route_random_filter():
    rng = np.random.default_rng(21)
    S, K = 5, 3
    F = rng.standard_normal((S, S, S))
    H = rng.standard_normal((4, 5, 3))
    a, b, g = rot_field(H.shape, 22)
    for brute, fft in ((O3.ext_corr3d_brute, O3.ext_corr3d_fft), (O3.ext_conv3d_brute, O3.ext_conv3d_fft)):
        yb, yf = brute(H, a, b, g, F, K), fft(H, a, b, g, F, K)
        assert np.max(np.abs(yb - yf)) <= 1e-10 * np.max(np.abs(yb))


def test_identity_field_is_plain_correlation_with_the_band_limited_filter():
    rng = np.random.default_rng(31)
    S, K = 5, 2
    F = rng.standard_normal((S, S, S))
    H = rng.standard_normal((6, 5, 4))
    z0 = np.zeros(H.shape)
    Ft = O3.rotated_band_limited(F, K, np.eye(3))
    ref = ndimage.correlate(H, Ft, mode="constant", cval=0.0)
    got = O3.ext_corr3d_fft(H, z0, z0, z0, F, K)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
