"""Pins of the float64 oracle (rotation group) against facts fixed by the paper and by
mathematics, independent of the oracle's own formulas. CPU only."""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.ndimage as nd
import scipy.signal as ss

import oracle as O
from synthetic import blurred_noise, random_filter, theta_field


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _polar(S):
    R = (S - 1) // 2
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    r = np.hypot(xx, yy)
    phi = np.arctan2(yy, xx)
    disk = (xx * xx + yy * yy) <= R * R
    return R, xx, yy, r, phi, disk


def _analytic_comps(S, kfun, K):
    """Component stack k = -K..K from an analytic radial/angular description:
    kfun(k, r) gives f_k(r); F_k(x) = f_k(|x|) e^{i k phi(x)} on the disk."""
    R, xx, yy, r, phi, disk = _polar(S)
    comps = np.zeros((2 * K + 1, S, S), complex)
    for k in range(-K, K + 1):
        comps[k + K] = np.where(disk, kfun(k, r) * np.exp(1j * k * phi), 0.0)
    return comps


# ---------------------------------------------------------------- decomposition pins

def test_bilinear_matches_library_interpolation():
    F = random_filter(11, 5, 3.0).astype(np.float64)
    rng = np.random.default_rng(1)
    dx = rng.uniform(-7, 7, 500)
    dy = rng.uniform(-7, 7, 500)
    ref = nd.map_coordinates(F, [dy + 5, dx + 5], order=1, mode="constant", cval=0.0)
    # map_coordinates treats the region between the last sample and the border as
    # constant-padded with a half-pixel ramp; compare where all four corners exist
    inside = (dx > -5) & (dx < 5) & (dy > -5) & (dy < 5)
    assert np.allclose(O.bilinear(F, dx, dy)[inside], ref[inside], atol=1e-13)
    # at integer offsets bilinear interpolation returns the grid value
    assert O.bilinear(F, 2.0, -3.0) == pytest.approx(F[5 - 3, 5 + 2], abs=1e-15)


def test_angular_sample_counts():
    assert O.default_angular_samples(8, 7) == 256
    assert O.default_angular_samples(16, 15) == 512
    assert O.default_angular_samples(16, 31) == 1024
    assert O.default_angular_samples(12, 10) == 256


def test_radial_profile_is_the_angular_fourier_integral():
    """f_k(rho) from the M-point rule converges to (1/2pi) int F(rho, phi) e^{-ik phi} dphi;
    quadrature of the library bilinear interpolant pins the DFT sign and scale."""
    F = random_filter(9, 7, 3.0).astype(np.float64)
    K = 3
    comps, f = O.angular_components(F, K, M=1 << 14)
    for d2 in (1, 5, 13):
        rho = np.sqrt(d2)

        def samp(phi):
            return nd.map_coordinates(F, [[4 + rho * np.sin(phi)], [4 + rho * np.cos(phi)]],
                                      order=1, mode="constant")[0]
        for k in (-2, 1, 3):
            # the interpolant has kinks where the circle crosses grid lines; tell quad
            kinks = []
            for g in range(-4, 5):
                if abs(g) <= rho:
                    a = np.arccos(g / rho)
                    b = np.arcsin(g / rho)
                    kinks += [a % (2 * np.pi), (-a) % (2 * np.pi), b % (2 * np.pi), (np.pi - b) % (2 * np.pi)]
            kinks = sorted(set(np.round(kinks, 12)))
            re = si.quad(lambda t: samp(t) * np.cos(k * t), 0, 2 * np.pi, points=kinks, limit=400)[0]
            im = si.quad(lambda t: -samp(t) * np.sin(k * t), 0, 2 * np.pi, points=kinks, limit=400)[0]
            ref = (re + 1j * im) / (2 * np.pi)
            assert abs(f[d2][k + K] - ref) < 1e-6


def test_decomposition_of_quarter_turned_filter():
    """np.rot90 maps F(x) to F(Qx), Q(dx, dy) = (-dy, dx): the filter rotated by -pi/2,
    so every component must pick up e^{-ik(-pi/2)} = i^k exactly (M divisible by 4)."""
    F = random_filter(15, 3, 4.0)
    K = 8
    c0, _ = O.angular_components(F, K)
    c1, _ = O.angular_components(np.rot90(F), K)
    ks = np.arange(-K, K + 1)
    assert np.allclose(c1, (1j ** ks)[:, None, None] * c0, atol=1e-13)


def test_full_band_components_reproduce_axis_pixels():
    """DFT inversion: with every angular frequency kept (k = -M/2+1..M/2-1 plus the
    Nyquist term), the components sum to the polar sample at each sample angle. On the
    axis pixels the sample angle is a grid direction and the bilinear sample is the
    grid value itself, so the sum must return F there."""
    S = 13
    R = 6
    F = random_filter(S, 8, 3.0)
    M = 64
    Kfull = M // 2 - 1
    comps, _ = O.angular_components(F, Kfull, M=M)
    recon = comps.sum(axis=0)
    phis = 2 * np.pi * np.arange(M) / M
    for d in range(1, R + 1):
        v = O.bilinear(F, d * np.cos(phis), d * np.sin(phis))
        c_nyq = np.sum(v * (-1.0) ** np.arange(M)) / M
        for m0, (dx, dy) in ((0, (d, 0)), (M // 4, (0, d)), (M // 2, (-d, 0)), (3 * M // 4, (0, -d))):
            total = recon[R + dy, R + dx] + c_nyq * (-1.0) ** m0
            assert total == pytest.approx(float(F[R + dy, R + dx]), abs=1e-12)


# ---------------------------------------------------------------- rotation convention pins

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                    "rotation_coefficient_matrices.txt")
_EV_NS = {"cos": np.cos, "sin": np.sin, "exp": np.exp}


def _ev(expr, **names):
    return eval(expr, {"__builtins__": {}, **_EV_NS}, names)


def _golden_examples():
    """Blocks of the fixture: {'basis': [expr in phi], 'rows': [[expr in T]]}."""
    blocks, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("basis:"):
            cur = {"basis": [e.strip() for e in line[len("basis:"):].split(",")], "rows": []}
            blocks.append(cur)
        else:
            cur["rows"].append([e.strip() for e in line.split(",")])
    return blocks


def test_golden_fixture_shape():
    ex = _golden_examples()
    assert [len(b["basis"]) for b in ex] == [1, 3, 3]
    assert all(len(b["rows"]) == len(b["basis"]) and all(len(r) == len(b["basis"]) for r in b["rows"])
               for b in ex)


@pytest.mark.parametrize("block", [0, 1, 2])
def test_rotation_matches_printed_matrices(block):
    """Sec. 3 prints, for three small bases, the matrix by which a rotation by Theta maps a
    filter's coefficient vector. A filter prof(r) * sum_j a_j basis_j(phi) is split into
    angular components by the plain angular DFT of its (band-limited) angular factor; the
    oracle's rotated filter sum_k e^{-ik Theta} F_k must equal the same profile with the
    coefficients (printed matrix) @ a."""
    ex = _golden_examples()[block]
    S = 15
    R, xx, yy, r, phi, disk = _polar(S)
    prof = np.exp(-r ** 2 / 18.0) * (1.0 + r)
    n = len(ex["basis"])
    rng = np.random.default_rng(block)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    K, M = 3, 64
    phis = 2 * np.pi * np.arange(M) / M
    ang = sum(a[j] * _ev(ex["basis"][j], phi=phis) for j in range(n))
    comps = np.zeros((2 * K + 1, S, S), complex)
    for k in range(-K, K + 1):
        ck = np.mean(ang * np.exp(-1j * k * phis))
        comps[k + K] = np.where(disk, prof * ck * np.exp(1j * k * phi), 0)
    for T in (0.3, 1.1, 2.5, -0.9):
        mat = np.array([[_ev(e, T=T) for e in row] for row in ex["rows"]], complex)
        b = mat @ a
        ref = np.where(disk, prof * sum(b[j] * _ev(ex["basis"][j], phi=phi) for j in range(n)), 0)
        assert np.allclose(O.rotated_filter(comps, T), ref, atol=1e-12)


# ---------------------------------------------------------------- extended operators

@pytest.fixture(scope="module")
def small_case():
    H = blurred_noise((26, 21), 0).astype(np.float64)
    F = random_filter(7, 1, 2.0)
    th = theta_field((26, 21), 2).astype(np.float64)
    comps, _ = O.angular_components(F, 3)
    return H, th, comps


def test_brute_equals_fft_route(small_case):
    H, th, comps = small_case
    assert rel(O.ext_corr_fft(H, th, comps), O.ext_corr_brute(H, th, comps)) < 1e-12
    assert rel(O.ext_conv_fft(H, th, comps), O.ext_conv_brute(H, th, comps)) < 1e-12
    # any FFT size at or above N + R gives the same zero-boundary result
    assert rel(O.ext_corr_fft(H, th, comps, P=(40, 33)), O.ext_corr_brute(H, th, comps)) < 1e-12


def test_real_filter_half_form(small_case):
    H, th, comps = small_case
    half = O.half_components(comps)
    full = O.ext_corr_fft(H, th, comps)
    assert np.max(np.abs(full.imag)) < 1e-12 * np.max(np.abs(full))
    assert rel(O.ext_corr_half(H, th, half), full.real) < 1e-12
    assert rel(O.ext_conv_half(H, th, half), O.ext_conv_fft(H, th, comps).real) < 1e-12


def test_constant_field_is_textbook_correlation(small_case):
    H, _, comps = small_case
    for t0 in (0.0, 0.9, 4.0):
        Ft = O.rotated_filter(comps, t0)
        th = np.full(H.shape, t0)
        ref = ss.correlate2d(H, Ft, mode="same", boundary="fill")
        assert rel(O.ext_corr_brute(H, th, comps), ref) < 1e-12
        refc = ss.convolve2d(H, Ft, mode="same", boundary="fill")
        assert rel(O.ext_conv_brute(H, th, comps), refc) < 1e-12


def test_steerable_derivative_of_gaussian_closed_form():
    """F = d/dx of a Gaussian has angular frequencies +-1 only, and its rotation by theta
    is cos(theta) G_x + sin(theta) G_y (Sec. 4.4, classical steering)."""
    S, sig = 13, 2.0
    R, xx, yy, r, phi, disk = _polar(S)
    g = np.exp(-r ** 2 / (2 * sig ** 2))
    comps = _analytic_comps(S, lambda k, rr: (-(rr * np.exp(-rr ** 2 / (2 * sig ** 2))) / (2 * sig ** 2))
                            * (abs(k) == 1), 1)
    Gx = np.where(disk, -xx / sig ** 2 * g, 0)
    Gy = np.where(disk, -yy / sig ** 2 * g, 0)
    H = blurred_noise((30, 27), 3).astype(np.float64)
    th = theta_field((30, 27), 4).astype(np.float64)
    ref = (np.cos(th) * ss.correlate2d(H, Gx, mode="same") + np.sin(th) * ss.correlate2d(H, Gy, mode="same"))
    assert rel(O.ext_corr_brute(H, th, comps), ref) < 1e-12
    assert rel(O.ext_corr_fft(H, th, comps), ref) < 1e-12


def test_bandlimited_filter_reproduced_exactly_under_rotation():
    """For an analytic filter of angular band <= K, the component route equals direct
    correlation with the analytically rotated filter F(r, phi - theta(p)) (Sec. 4.3)."""
    S = 11
    R, xx, yy, r, phi, disk = _polar(S)
    b1, b2 = 0.4, -1.2

    def Fan(rr, ph):
        return np.exp(-rr ** 2 / 10.0) * (0.3 + rr * np.cos(ph - b1) + 0.2 * rr ** 2 * np.cos(2 * (ph - b2)))

    def fk(k, rr):
        e = np.exp(-rr ** 2 / 10.0)
        return {0: 0.3 * e, 1: 0.5 * rr * e * np.exp(-1j * b1), -1: 0.5 * rr * e * np.exp(1j * b1),
                2: 0.1 * rr ** 2 * e * np.exp(-2j * b2), -2: 0.1 * rr ** 2 * e * np.exp(2j * b2)}.get(k, 0 * rr)
    comps = _analytic_comps(S, fk, 2)
    comps[2, R, R] = Fan(0.0, 0.0)
    H = blurred_noise((17, 19), 6).astype(np.float64)
    th = theta_field((17, 19), 7).astype(np.float64)
    ref = np.zeros(H.shape)
    Hp = np.pad(H, R)
    for i in range(H.shape[0]):
        for j in range(H.shape[1]):
            Fr = np.where(disk, Fan(r, phi - th[i, j]), 0)
            ref[i, j] = np.sum(Hp[i:i + S, j:j + S] * Fr)
    assert rel(O.ext_corr_brute(H, th, comps).real, ref) < 1e-12


def test_radial_filter_ignores_field(small_case):
    H, th, _ = small_case
    F = random_filter(7, 9, 2.0)
    comps, _ = O.angular_components(F, 0)
    a = O.ext_corr_brute(H, th, comps)
    b = O.ext_corr_brute(H, np.zeros_like(th), comps)
    assert rel(a, b) < 1e-14
    assert rel(O.ext_conv_brute(H, th, comps), O.ext_conv_brute(H, 3 + th, comps)) < 1e-14


def test_single_frequency_filter(small_case):
    """Sec. 3 example n = 1: correlate once, then multiply by e^{i k Theta(p)}."""
    H, th, _ = small_case
    S, k = 9, 3
    comps = _analytic_comps(S, lambda kk, rr: np.exp(-rr ** 2 / 6) * rr * (kk == k), k)
    Fk = comps[2 * k]
    ref = np.exp(1j * k * th) * ss.correlate2d(H, Fk, mode="same")
    assert rel(O.ext_corr_brute(H, th, comps), ref) < 1e-12


def test_delta_responses(small_case):
    """Sec. 2.3: a delta at q0 convolves to the filter transformed by T(q0) placed at
    q0; the correlation at p reads conj F_{theta(p)}(q0 - p)."""
    _, th, comps = small_case
    ny, nx = th.shape
    R = (comps.shape[1] - 1) // 2
    q0 = (11, 9)
    H = np.zeros((ny, nx))
    H[q0] = 1.0
    y = O.ext_conv_brute(H, th, comps)
    Ft = O.rotated_filter(comps, th[q0])
    ref = np.zeros((ny, nx), complex)
    ref[q0[0] - R:q0[0] + R + 1, q0[1] - R:q0[1] + R + 1] = Ft
    assert np.allclose(y, ref, atol=1e-14)
    yc = O.ext_corr_brute(H, th, comps)
    refc = np.zeros((ny, nx), complex)
    for i in range(ny):
        for j in range(nx):
            dy, dx = q0[0] - i, q0[1] - j
            if abs(dy) <= R and abs(dx) <= R:
                refc[i, j] = np.conj(O.rotated_filter(comps, th[i, j])[R + dy, R + dx])
    assert np.allclose(yc, refc, atol=1e-14)


def test_quarter_turn_equivariance():
    """Rotating the signal and field by 90 degrees on the grid (np.rot90) and shifting
    the field by -pi/2 rotates the output the same way, exactly."""
    n = 20
    H = blurred_noise((n, n), 11).astype(np.float64)
    th = theta_field((n, n), 12).astype(np.float64)
    comps, _ = O.angular_components(random_filter(9, 13, 2.5), 4)
    for f in (O.ext_corr_brute, O.ext_conv_brute):
        a = f(np.rot90(H), np.rot90(th) - np.pi / 2, comps)
        b = np.rot90(f(H, th, comps))
        assert rel(a, b) < 1e-13


def test_linearity(small_case):
    H, th, comps = small_case
    H2 = blurred_noise(H.shape, 21).astype(np.float64)
    a, b = 0.7, -1.9
    assert rel(O.ext_corr_brute(a * H + b * H2, th, comps),
               a * O.ext_corr_brute(H, th, comps) + b * O.ext_corr_brute(H2, th, comps)) < 1e-13
    c = 0.4 - 1.1j
    assert rel(O.ext_corr_brute(H, th, c * comps), np.conj(c) * O.ext_corr_brute(H, th, comps)) < 1e-13
    assert rel(O.ext_conv_brute(H, th, c * comps), c * O.ext_conv_brute(H, th, comps)) < 1e-13


def test_convolution_is_adjoint_of_correlation(small_case):
    """Scatter/gather duality: <conv_F(H), g> = <H, corr_F(g)> for a real filter."""
    H, th, comps = small_case
    g = np.random.default_rng(5).standard_normal(H.shape)
    lhs = np.sum(O.ext_conv_brute(H, th, comps).real * g)
    rhs = np.sum(H * O.ext_corr_brute(g, th, comps).real)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_matching_is_correlation_at_each_angle(small_case):
    H, _, comps = small_case
    A = 16
    score, idx, C = O.match_rotations(H, comps, n_angles=A)
    for m in (0, 5, 11):
        ref = O.ext_corr_brute(H, np.full(H.shape, 2 * np.pi * m / A), comps).real
        assert rel(C[m], ref) < 1e-12
    assert np.array_equal(score, C.max(axis=0))
    assert np.all(C[idx, np.arange(H.shape[0])[:, None], np.arange(H.shape[1])] == score)


def test_matching_finds_planted_pattern():
    """A disk pattern pasted at a known angle peaks near its true position and angle."""
    from synthetic import _bilinear_sample
    S = 15
    R = 7
    rng = np.random.default_rng(3)
    pat = nd.gaussian_filter(rng.standard_normal((S, S)), 1.0)
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    disk = xx ** 2 + yy ** 2 <= R * R
    pat = np.where(disk, pat - pat[disk].mean(), 0)
    img = 0.02 * np.random.default_rng(4).standard_normal((48, 48))
    a = 2 * np.pi * 10 / 32
    ca, sa = np.cos(a), np.sin(a)
    vals = _bilinear_sample(pat, -sa * xx + ca * yy + R, ca * xx + sa * yy + R)
    img[20 - R:20 + R + 1, 27 - R:27 + R + 1][disk] = vals[disk]
    comps, _ = O.angular_components(pat, 7)
    score, idx, _ = O.match_rotations(img, comps, n_angles=32)
    i, j = np.unravel_index(np.argmax(score), score.shape)
    assert (i, j) == (20, 27)
    assert abs(int(idx[i, j]) - 10) <= 1
