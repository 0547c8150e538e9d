"""Normalised filtering (Sec. 8, eq. normalization) through ecc_normalized_convolution
against the float64 oracle: line-integral convolution of white noise with a long, narrow
anisotropic Gaussian rotated by a vortex field, both strategies, ragged shapes, batches,
the full 1024 x 1024 workload, constant images, and scale plans (the same call as the
scale smoothing). Tolerance: rel-L2 and rel-inf <= 1e-5."""
import numpy as np
import pytest

import oracle as O
from synthetic import anisotropic_gaussian, lic_config, scale_field, blurred_noise, vortex_field

pytestmark = pytest.mark.gpu
TOL = 1e-5
TWO_PASS, TILED = 1, 2


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def E():
    import torch
    import paper_2006_13188_amd as E_
    assert torch.cuda.is_available()
    E_.lib()
    return E_


@pytest.fixture(scope="module", params=[TWO_PASS, TILED], ids=["two_pass", "tiled"])
def sctx(E, request):
    c = E.Context(0)
    c.set_strategy(request.param)
    yield c, request.param
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_lic(img, theta, filt, K):
    comps, _ = O.angular_components(filt, K)
    y, _, _ = O.normalized_conv_half(img.astype(np.float64), theta.astype(np.float64), O.half_components(comps))
    return y


@pytest.mark.parametrize("shape,S,K", [((200, 333), 15, 8), ((97, 130), 31, 16), ((150, 151), 21, 12),
                                       ((64, 64), 9, 4)])
def test_lic_parity(E, sctx, shape, S, K):
    ctx, strat = sctx
    img = np.random.default_rng(60 + S).random(shape).astype(np.float32)
    th = vortex_field(shape, 61 + S, sigma=6.0)
    filt = anisotropic_gaussian(S, S / 4.0, 1.2)
    print(f"lic strategy={strat} shape={shape} S={S} K={K}", flush=True)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    got = host(E.ecc_normalized_convolution(ctx, plan, dev(img), dev(th))).astype(np.float64)
    ref = oracle_lic(img, th, filt, K)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    plan.close()


@pytest.fixture(scope="module")
def actx(E):
    c = E.Context(0)   # AUTO: block side >= the filter diameter
    yield c
    c.close()


@pytest.mark.parametrize("shape,S,K", [((200, 230), 53, 12), ((130, 97), 65, 16), ((301, 263), 61, 20)])
def test_lic_parity_overlap_add_blocks(E, actx, shape, S, K):
    """Radii above 24 under the default strategy: 128-point blocks, so the overlap-add
    ratio kernel runs (rotation components of odd parity: imaginary spectra); the same
    components without parity take the two launches of the block convolution."""
    img = np.random.default_rng(62 + S).random(shape).astype(np.float32)
    th = vortex_field(shape, 63 + S, sigma=6.0)
    filt = anisotropic_gaussian(S, S / 4.0, 1.5)
    print(f"lic overlap-add shape={shape} S={S} K={K}", flush=True)
    plan = E.FilterPlan.rotation(actx, dev(filt), K)
    strat, n, T = actx.describe(E.CONVOLUTION, plan, *shape)
    assert strat == TILED and n == 128
    assert actx.workspace_size(E.WS_NORMALIZED_CONVOLUTION, plan, *shape) == \
        (-(-shape[0] // T)) * (-(-shape[1] // T)) * 128 * 128 * 8
    got = host(E.ecc_normalized_convolution(actx, plan, dev(img), dev(th))).astype(np.float64)
    ref = oracle_lic(img, th, filt, K)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    gplan = E.FilterPlan.from_components(actx, plan.components())
    got2 = host(E.ecc_normalized_convolution(actx, gplan, dev(img), dev(th))).astype(np.float64)
    assert rel2(got2, ref) <= TOL and relinf(got2, ref) <= TOL
    gplan.close()
    plan.close()


def test_lic_batch_overlap_add_blocks(E, actx):
    B, shape, S, K = 2, (150, 170), 57, 10
    imgs = np.stack([np.random.default_rng(75 + b).random(shape) for b in range(B)]).astype(np.float32)
    ths = np.stack([vortex_field(shape, 85 + b, sigma=5.0) for b in range(B)])
    filt = anisotropic_gaussian(S, 12.0, 1.5)
    plan = E.FilterPlan.rotation(actx, dev(filt), K)
    got = host(E.ecc_normalized_convolution(actx, plan, dev(imgs), dev(ths))).astype(np.float64)
    for b in range(B):
        ref = oracle_lic(imgs[b], ths[b], filt, K)
        assert rel2(got[b], ref) <= TOL and relinf(got[b], ref) <= TOL
    plan.close()


def test_lic_batch(E, sctx):
    ctx, strat = sctx
    B, shape, S, K = 3, (120, 140), 15, 8
    imgs = np.stack([np.random.default_rng(70 + b).random(shape) for b in range(B)]).astype(np.float32)
    ths = np.stack([vortex_field(shape, 80 + b, sigma=5.0) for b in range(B)])
    filt = anisotropic_gaussian(S, 4.0, 1.0)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    got = host(E.ecc_normalized_convolution(ctx, plan, dev(imgs), dev(ths))).astype(np.float64)
    for b in range(B):
        ref = oracle_lic(imgs[b], ths[b], filt, K)
        assert rel2(got[b], ref) <= TOL and relinf(got[b], ref) <= TOL
    plan.close()


def test_constant_image_is_preserved(E, sctx):
    ctx, _ = sctx
    shape = (180, 211)
    th = vortex_field(shape, 90, sigma=6.0)
    plan = E.FilterPlan.rotation(ctx, dev(anisotropic_gaussian(31, 8.0, 1.5)), 16)
    got = host(E.ecc_normalized_convolution(ctx, plan, dev(np.full(shape, 0.625, np.float32)), dev(th)))
    assert np.max(np.abs(got - 0.625)) <= 1e-5 * 0.625
    plan.close()


def test_full_size_lic(E, sctx):
    """The line-integral-convolution workload: 1024 x 1024 white noise, 31 x 31 Gaussian
    (sigma 8 along, 1.5 across), K = 16, vortex field."""
    ctx, strat = sctx
    img, filt, th = lic_config()
    print(f"lic full size strategy={strat}", flush=True)
    plan = E.FilterPlan.rotation(ctx, dev(filt), 16)
    got = host(E.ecc_normalized_convolution(ctx, plan, dev(img), dev(th))).astype(np.float64)
    ref = oracle_lic(img, th, filt, 16)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    plan.close()


def test_scale_plan_is_the_scale_smoothing(E, sctx):
    """For a scale plan the call divides the signal by s^2: the same kernels and values as
    ecc_scale_smooth."""
    ctx, _ = sctx
    shape = (150, 170)
    img = blurred_noise(shape, 95)
    s = scale_field(shape, 96, 1.0, 3.0, sigma=6.0)
    plan = E.FilterPlan.scale(ctx, sigma0=1.0, scale_min=1.0, scale_max=3.0, components=24)
    a = host(E.ecc_normalized_convolution(ctx, plan, dev(img), dev(s)))
    b = host(E.ecc_scale_smooth(ctx, plan, dev(img), dev(s)))
    assert np.array_equal(a, b)
    plan.close()


# ---------------------------------------------------------------- matrix-core precisions

PREC_TOL = {1: (1e-5, 1e-5), 2: (1e-4, 1e-4)}   # (rel-L2, rel-inf): float16 hi/lo, bfloat16 hi/lo (2^-16 operands)


@pytest.mark.parametrize("prec", [1, 2], ids=["fp16_hilo", "bf16_hilo"])
def test_lic_matrix_core_precisions(E, actx, prec):
    """The overlap-add kernel's radix-16 passes on the matrix cores (hi/lo operands): LIC
    with a 65 x 65 filter against the float64 oracle."""
    shape, S, K = (300, 280), 65, 12
    img = np.random.default_rng(1).random(shape).astype(np.float32)
    th = vortex_field(shape, 2, sigma=6.0)
    filt = anisotropic_gaussian(S, 14.0, 2.0)
    plan = E.FilterPlan.rotation(actx, dev(filt), K)
    got = host(E.ecc_normalized_convolution(actx, plan, dev(img), dev(th), precision=prec)).astype(np.float64)
    ref = oracle_lic(img, th, filt, K)
    t2, ti = PREC_TOL[prec]
    assert rel2(got, ref) <= t2 and relinf(got, ref) <= ti, (rel2(got, ref), relinf(got, ref))
    plan.close()


@pytest.mark.parametrize("prec", [1, 2], ids=["fp16_hilo", "bf16_hilo"])
def test_scale_smoothing_matrix_core_full_size(E, actx, prec):
    """The scale-group workload (2048 x 2048, 24 components, 65 x 65 support) with the
    matrix-core passes, against the float64 oracle."""
    from synthetic import scale_config
    img, s = scale_config(2048)
    print(f"scale smoothing 2048^2 precision={prec}", flush=True)
    plan = E.FilterPlan.scale(actx)
    got = host(E.ecc_scale_smooth(actx, plan, dev(img), dev(s), precision=prec)).astype(np.float64)
    ref = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), O.ScaleParams())[0]
    t2, ti = PREC_TOL[prec]
    assert rel2(got, ref) <= t2 and relinf(got, ref) <= ti, (rel2(got, ref), relinf(got, ref))
    plan.close()


def test_matrix_core_precisions_need_the_overlap_add_kernel(E, actx):
    plan = E.FilterPlan.rotation(actx, dev(anisotropic_gaussian(31, 8.0, 1.5)), 16)
    img = dev(np.ones((128, 128), np.float32))
    with pytest.raises(E.EccError) as ei:
        E.ecc_normalized_convolution(actx, plan, img, img, precision=1)
    assert ei.value.status == 2
    plan.close()
