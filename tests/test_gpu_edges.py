"""Edge cases of the forward operators on the GPU against the float64 oracle.

* the largest accepted image side (4096 x 4096, 31 x 31 filter, K = 16) with the
  block strategy (default and forced): pixels at the corners, on block seams and at
  random, each summed by the oracle's brute-force definition on the part of the image it
  depends on; the two-pass strategy, whose row transforms stop at 4096 points, reports
  UNSUPPORTED there and runs at 4000 x 4000 (transform length 4032);
* the smallest images a filter plan accepts (a 3 x 3 filter on images 3 pixels wide or
  high) and 1 x 1 filters built from components on 1 x 1 and 2 x 5 images, every pixel
  against the oracle;
* sizes outside the documented limits (empty images, sides above 4096) rejected with
  an error before anything is enqueued.

Tolerance as in the other parity tests: max|y - y_ref| / max|y_ref| <= 1e-5 (float32
path against the float64 oracle)."""
import numpy as np
import pytest

import oracle as O
from synthetic import scale_field, blurred_noise, random_filter, theta_field

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def E():
    import torch
    import paper_2006_13188_amd as E_
    assert torch.cuda.is_available()
    E_.lib()  # fails loudly if the library is missing
    return E_


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def strategies(E):
    return [("tiled", E.STRATEGY_TILED), ("two_pass", E.STRATEGY_TWO_PASS)]


def brute_at(op, img, theta, comps, i, j, R):
    """y(i, j) by the definition: the oracle's brute force on the rows and columns within
    R of the pixel (zero outside the image, so cropping there changes nothing)."""
    ny, nx = img.shape
    i0, i1 = max(0, i - R), min(ny, i + R + 1)
    j0, j1 = max(0, j - R), min(nx, j + R + 1)
    f = O.ext_corr_brute if op == 0 else O.ext_conv_brute
    y = f(img[i0:i1, j0:j1].astype(np.float64), theta[i0:i1, j0:j1].astype(np.float64), comps)
    return float(y[i - i0, j - j0].real)


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_maximum_image_side(E, op):
    n, S, K = 4096, 31, 16
    R = (S - 1) // 2
    img = blurred_noise((n, n), 31)
    theta = theta_field((n, n), 32)
    filt = random_filter(S, 33, 4.0 * S / 15)
    comps, _ = O.angular_components(filt, K)
    rng = np.random.default_rng(5)
    pts = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (63, 64), (64, 63), (2047, 2048),
           (n - 1, 1000), (1000, n - 1)] + [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(12)]
    # two-pass: transforms of 4126 points; the convolution's row kernels take them, the
    # correlation's combined inverse row kernel refuses rows above 4096 points (its
    # 4000-pixel sub-image is checked instead)
    cases = [("auto", E.STRATEGY_AUTO, n), ("tiled", E.STRATEGY_TILED, n),
             ("two_pass", E.STRATEGY_TWO_PASS, 4000 if op == 0 else n)]
    for name, strat, m in cases:
        sub = [(i, j) for (i, j) in pts if i < m and j < m] + [(m - 1, m - 1), (0, m - 1)]
        refs = {p: brute_at(op, img[:m, :m], theta[:m, :m], comps, p[0], p[1], R) for p in sub}
        ctx = E.Context(0)
        try:
            ctx.set_strategy(strat)
            plan = E.FilterPlan.rotation(ctx, dev(filt), K)
            if strat == E.STRATEGY_TWO_PASS and op == 0:
                assert ctx.fft_size(n, R) > 4096
                with pytest.raises(E.EccError) as ei:
                    E.ecc_extended(ctx, op, plan, dev(img), dev(theta))
                assert ei.value.status == 2   # ECC_ERR_UNSUPPORTED
            y = host(E.ecc_extended(ctx, op, plan, dev(img[:m, :m]), dev(theta[:m, :m]))).astype(np.float64)
            plan.close()
        finally:
            ctx.close()
        assert np.all(np.isfinite(y)), name
        scale = np.max(np.abs(y))
        for (i, j), ref in refs.items():
            assert abs(y[i, j] - ref) <= TOL * scale, (name, i, j, y[i, j], ref)


@pytest.mark.parametrize("shape", [(3, 3), (3, 200), (200, 3), (5, 4)])
@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_smallest_images(E, op, shape):
    img = blurred_noise(shape, 41, sigma=0.8)
    theta = theta_field(shape, 42, sigma=1.0)
    filt = random_filter(3, 43, 1.0)
    K = 2
    comps, _ = O.angular_components(filt, K)
    half = O.half_components(comps)
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    ref = f(img.astype(np.float64), theta.astype(np.float64), half)
    for name, strat in strategies(E):
        ctx = E.Context(0)
        try:
            ctx.set_strategy(strat)
            plan = E.FilterPlan.rotation(ctx, dev(filt), K)
            y = host(E.ecc_extended(ctx, op, plan, dev(img), dev(theta))).astype(np.float64)
            plan.close()
        finally:
            ctx.close()
        assert relinf(y, ref) <= TOL, (name, relinf(y, ref))


@pytest.mark.parametrize("shape", [(4, 40), (9, 6), (1, 1)])
def test_images_smaller_than_the_filter_radius(E, shape):
    """Scale smoothing (65 x 65 support, R = 32) of images with a side <= R: the two-pass
    transform size must hold the whole filter window (2R + 1 taps) as well as n + R; every
    strategy against the oracle."""
    img = blurred_noise(shape, 47, sigma=0.8) if min(shape) > 1 else np.array([[0.7]], np.float32)
    s = scale_field(shape, 48, 1.0, 8.0, sigma=1.0) if min(shape) > 1 else np.array([[3.0]], np.float32)
    ref, _, _ = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), O.ScaleParams())
    for name, strat in strategies(E) + [("auto", E.STRATEGY_AUTO)]:
        ctx = E.Context(0)
        try:
            ctx.set_strategy(strat)
            plan = E.FilterPlan.scale(ctx)
            try:
                y = host(E.ecc_scale_smooth(ctx, plan, dev(img), dev(s))).astype(np.float64)
            except E.EccError as err:       # a strategy without a block shape for R = 32 says so
                assert strat == E.STRATEGY_TILED and err.status == 2, (name, err)
                continue
            finally:
                plan.close()
        finally:
            ctx.close()
        assert relinf(y, ref) <= TOL, (name, relinf(y, ref))


@pytest.mark.parametrize("shape", [(1, 1), (2, 5)])
@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_one_pixel_filter_from_components(E, op, shape):
    """S = 1: y = Re sum_k w_k e^{ik theta} H conj(F_k(0)) (correlation) and
    Re sum_k w_k e^{-ik theta} H F_k(0) (convolution), any component values."""
    import torch
    rng = np.random.default_rng(44)
    half = (rng.standard_normal((4, 1, 1)) + 1j * rng.standard_normal((4, 1, 1))).astype(np.complex64)
    img = rng.standard_normal(shape).astype(np.float32)
    theta = (rng.random(shape) * 2 * np.pi).astype(np.float32)
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    ref = f(img.astype(np.float64), theta.astype(np.float64), half.astype(np.complex128))
    for name, strat in strategies(E):
        ctx = E.Context(0)
        try:
            ctx.set_strategy(strat)
            plan = E.FilterPlan.from_components(ctx, torch.from_numpy(half).cuda())
            y = host(E.ecc_extended(ctx, op, plan, dev(img), dev(theta))).astype(np.float64)
            plan.close()
        finally:
            ctx.close()
        assert relinf(y, ref) <= TOL, (name, relinf(y, ref))


def test_sizes_outside_the_limits_rejected(E):
    import torch
    ctx = E.Context(0)
    try:
        plan = E.FilterPlan.rotation(ctx, dev(random_filter(3, 45, 1.0)), 1)
        for shape in [(0, 8), (8, 0), (4097, 3), (3, 4097)]:
            img = torch.zeros(shape, dtype=torch.float32, device="cuda")
            out = torch.full(shape, 7.0, dtype=torch.float32, device="cuda")
            with pytest.raises(E.EccError):
                E.ecc_extended(ctx, 0, plan, img, img.clone(), out=out)
            assert torch.all(out == 7.0)
        plan.close()
    finally:
        ctx.close()
