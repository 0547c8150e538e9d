"""Both evaluation strategies of the extended correlation and convolution (and the
scale-group smoothing) against the float64 oracle.

TWO_PASS is the paper's whole-image FFT form; TILED evaluates overlap-save blocks on chip.
Each runs on its own context with the strategy forced, on shapes that span several
blocks with ragged edges, every supported block size (N = 64, 96, 128), the largest
radius that still has a block, batches, and the full 1024 x 1024 workload.
Tolerance as in test_gpu_rotation: rel-L2 and rel-inf <= 1e-5."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, random_filter, rotation_config, scale_field, theta_field

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
    return t.cpu().numpy()


def oracle_corr(img, filt, theta, K, op=0):
    comps, _ = O.angular_components(filt, K)
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    return f(img.astype(np.float64), theta.astype(np.float64), O.half_components(comps))


@pytest.mark.parametrize("shape,S,K", [
    ((128, 128), 15, 8),     # small workload: N = 64 blocks
    ((67, 93), 9, 3),
    ((200, 173), 21, 10),    # N = 96
    ((33, 33), 31, 12),      # one block larger than the image
    ((150, 211), 63, 16),    # R = 31: N = 128
    ((97, 130), 81, 6),      # R = 40: N = 128, T = 48 (tiled only when forced)
])
@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_forward_parity(E, sctx, op, shape, S, K):
    ctx, strat = sctx
    img = blurred_noise(shape, 5)
    filt = random_filter(S, 6, 4.0 * S / 15)
    theta = theta_field(shape, 7)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    used, n, blk = ctx.describe(op, plan, *shape)
    assert used == strat
    if strat == TILED:
        assert n in (64, 96, 128) and 16 <= blk <= n - (S - 1)
    y = host(E.ecc_extended(ctx, op, plan, dev(img), dev(theta))).astype(np.float64)
    ref = oracle_corr(img, filt, theta, K, op)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_batch(E, sctx, op):
    ctx, _ = sctx
    imgs = np.stack([blurred_noise((150, 131), 60 + i) for i in range(3)])
    ths = np.stack([theta_field((150, 131), 70 + i) for i in range(3)])
    filt = random_filter(17, 9, 4.5)
    plan = E.FilterPlan.rotation(ctx, dev(filt), 7)
    yb = host(E.ecc_extended(ctx, op, plan, dev(imgs), dev(ths)))
    for i in range(3):
        ref = oracle_corr(imgs[i], filt, ths[i], 7, op)
        assert rel2(yb[i].astype(np.float64), ref) <= TOL


def test_strided_rows(E, sctx):
    """Leading dimensions larger than the width (views into wider buffers)."""
    import torch
    ctx, _ = sctx
    img = blurred_noise((120, 100), 11)
    th = theta_field((120, 100), 12)
    filt = random_filter(13, 13, 3.5)
    plan = E.FilterPlan.rotation(ctx, dev(filt), 6)
    Hw = torch.zeros((120, 131), device="cuda")
    Tw = torch.zeros((120, 117), device="cuda")
    Ow = torch.full((120, 109), 5.0, device="cuda")
    Hw[:, :100] = dev(img)
    Tw[:, :100] = dev(th)
    E.ecc_extended(ctx, 0, plan, Hw[:, :100], Tw[:, :100], out=Ow[:, :100])
    y = host(Ow)
    ref = oracle_corr(img, filt, th, 6)
    assert rel2(y[:, :100].astype(np.float64), ref) <= TOL
    assert np.all(y[:, 100:] == 5.0)   # nothing written past nx


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_full_size(E, sctx, op):
    img, filt, theta, K = rotation_config(1024, 31, 16, seeds=(10, 11, 12))
    ctx, _ = sctx
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    y = host(E.ecc_extended(ctx, op, plan, dev(img), dev(theta))).astype(np.float64)
    ref = oracle_corr(img, filt, theta, K, op)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


def test_auto_choice_and_unsupported_radius(E):
    ctx = E.Context(0)
    try:
        plan = E.FilterPlan.rotation(ctx, dev(random_filter(31, 1, 8.0)), 16)
        assert ctx.describe(0, plan, 1024, 1024) == (TILED, 96, 64)
        assert ctx.describe(1, plan, 1024, 1024)[0] == TILED      # convolution
        big = E.FilterPlan.rotation(ctx, dev(random_filter(121, 2, 30.0)), 4)   # R = 60
        assert ctx.describe(0, big, 300, 300)[0] == TWO_PASS
        ctx.set_strategy(TILED)
        img = dev(blurred_noise((300, 300), 3))
        with pytest.raises(E.EccError):
            E.ecc_extended(ctx, 0, big, img, img)
    finally:
        ctx.close()


def test_context_close_with_live_plans(E):
    """Closing a context also closes its plans; later calls on other contexts are clean."""
    ctx = E.Context(0)
    plan = E.FilterPlan.rotation(ctx, dev(random_filter(9, 3, 2.0)), 3)
    ctx.close()
    assert plan.h is None
    plan.close()   # no-op
    ctx2 = E.Context(0)
    try:
        img, filt, theta, K = rotation_config(64, 9, 3)
        p2 = E.FilterPlan.rotation(ctx2, dev(filt), K)
        y = host(E.ecc_extended(ctx2, 0, p2, dev(img), dev(theta))).astype(np.float64)
        assert rel2(y, oracle_corr(img, filt, theta, K)) <= TOL
    finally:
        ctx2.close()


SMALLP = dict(sigma0=1.0, scale_min=1.0, scale_max=2.0, components=12, period_factor=1.5)


@pytest.mark.parametrize("shape", [(64, 80), (141, 97)])
def test_scale_smooth_parity(E, sctx, shape):
    """Ratio form of the scale-adaptive smoothing (two signals sharing the phases)."""
    ctx, _ = sctx
    plan = E.FilterPlan.scale(ctx, **SMALLP)
    img = blurred_noise(shape, 30)
    s = scale_field(shape, 31, 1.0, 2.0, sigma=4.0)
    y = host(E.ecc_scale_smooth(ctx, plan, dev(img), dev(s))).astype(np.float64)
    ref, _, _ = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), O.ScaleParams(1.0, 1.0, 2.0, 12, 1.5))
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


def test_scale_extended_convolution(E, sctx):
    ctx, _ = sctx
    plan = E.FilterPlan.scale(ctx, **SMALLP)
    img = blurred_noise((120, 90), 33)
    s = scale_field((120, 90), 34, 1.0, 2.0, sigma=3.0)
    y = host(E.ecc_extended(ctx, E.CONVOLUTION, plan, dev(img), dev(s))).astype(np.float64)
    comps, w, om1 = O.scale_components(O.ScaleParams(1.0, 1.0, 2.0, 12, 1.5))
    ref = O.ext_conv_half(img.astype(np.float64), om1 * np.log(s.astype(np.float64)), comps, w)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL


@pytest.fixture(scope="module")
def scale_full():
    from synthetic import scale_config
    img, s = scale_config(2048)
    ref, _, _ = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), O.ScaleParams())
    return img, s, ref


def test_scale_full_size(E, sctx, scale_full):
    """2048^2 scale-adaptive smoothing, 24 components (65 x 65 support), s in [1, 8]."""
    ctx, _ = sctx
    img, s, ref = scale_full
    plan = E.FilterPlan.scale(ctx)
    y = host(E.ecc_scale_smooth(ctx, plan, dev(img), dev(s))).astype(np.float64)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


def test_tiled_symmetric_and_general_pair_forms(E):
    """At N = 96 a rotation plan runs the symmetric pair form (centred block spectra, one
    set of spectrum loads per item and its mirror) and a plan built from the same
    components runs the general pair form (no parity assumed): both match the oracle, on a
    shape with ragged blocks and an odd number of components."""
    ctx = E.Context(0)
    ctx.set_strategy(TILED)
    try:
        S, K = 31, 10
        filt = random_filter(S, 32, 4.0 * S / 15)
        plan_r = E.FilterPlan.rotation(ctx, dev(filt), K)
        plan_c = E.FilterPlan.from_components(ctx, plan_r.components())
        # a shape with ragged blocks that the chooser runs with N = 96 transforms
        shapes = [sh for sh in ((520, 491), (700, 653), (1024, 1000))
                  if ctx.describe(0, plan_r, *sh)[1] == 96]
        assert shapes, "no candidate shape runs N = 96 blocks"
        shape = shapes[0]
        assert ctx.describe(0, plan_r, *shape)[1:] == ctx.describe(0, plan_c, *shape)[1:]
        img = blurred_noise(shape, 31)
        theta = theta_field(shape, 33)
        ref = oracle_corr(img, filt, theta, K)
        for plan in (plan_r, plan_c):
            y = host(E.ecc_extended(ctx, 0, plan, dev(img), dev(theta))).astype(np.float64)
            assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))
        plan_r.close()
        plan_c.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("source", ["rotation_plan", "from_components"])
def test_adjoint_at_n96_blocks_both_strategies(E, source):
    """The convolution adjoint where the block strategy runs N = 96 transforms (radius
    15): the signal and field parts as a tiled correlation with a second output (the
    symmetric pair form for a rotation plan, the general form for a plan built from
    components) and the filter part as per-block lag sums, and the two-pass adjoint on
    the same input; every gradient against the float64 oracle."""
    import torch
    cts = [E.Context(0), E.Context(0)]
    cts[0].set_strategy(TILED)
    cts[1].set_strategy(TWO_PASS)
    try:
        S, K = 31, 6
        filt = random_filter(S, 41, 4.0 * S / 15)
        half = O.half_components(O.angular_components(filt, K)[0])
        if source == "rotation_plan":
            plans = [E.FilterPlan.rotation(c, dev(filt), K) for c in cts]
        else:
            half = half.astype(np.complex64).astype(np.complex128)
            plans = [E.FilterPlan.from_components(c, torch.from_numpy(half.astype(np.complex64)).cuda())
                     for c in cts]
        shapes = [sh for sh in ((520, 491), (700, 653), (1024, 1000))
                  if cts[0].describe(0, plans[0], *sh)[1] == 96]
        assert shapes, "no candidate shape runs N = 96 blocks"
        shape = shapes[0]
        img = blurred_noise(shape, 42)
        th = theta_field(shape, 43)
        g = np.random.default_rng(44).standard_normal(shape).astype(np.float32)
        outs = []
        for c, p in zip(cts, plans):
            gs, gc, gf = E.ecc_extended_backward(c, p, dev(img[None]), dev(th[None]), dev(g[None]))
            outs.append((host(gs)[0].astype(np.float64), host(gf)[0].astype(np.float64),
                         host(gc).astype(np.complex128)))
        for p in plans:
            p.close()
    finally:
        for c in cts:
            c.close()
    rh, rt, rc = O.conv_backward(img.astype(np.float64), th.astype(np.float64), half, g.astype(np.float64))
    for gs, gf, gc in outs:
        assert rel2(gs, rh) <= TOL and relinf(gs, rh) <= 2 * TOL, (rel2(gs, rh), relinf(gs, rh))
        assert rel2(gf, rt) <= TOL and relinf(gf, rt) <= 2 * TOL, (rel2(gf, rt), relinf(gf, rt))
        assert rel2(gc, rc) <= TOL, rel2(gc, rc)


@pytest.mark.parametrize("K", [0, 1, 2])
def test_tiled_symmetric_pair_form_few_components(E, K):
    """The symmetric pair form with one component (K = 0: only the first half of a pair),
    two (one full pair) and three (a pair and a half pair), against the oracle."""
    ctx = E.Context(0)
    ctx.set_strategy(TILED)
    try:
        S = 31
        filt = random_filter(S, 50 + K, 4.0 * S / 15)
        plan = E.FilterPlan.rotation(ctx, dev(filt), K)
        shapes = [sh for sh in ((520, 491), (700, 653), (1024, 1000))
                  if ctx.describe(0, plan, *sh)[1] == 96]
        assert shapes, "no candidate shape runs N = 96 blocks"
        shape = shapes[0]
        img = blurred_noise(shape, 60 + K)
        theta = theta_field(shape, 70 + K)
        y = host(E.ecc_extended(ctx, 0, plan, dev(img), dev(theta))).astype(np.float64)
        ref = oracle_corr(img, filt, theta, K)
        assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))
        plan.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_two_pass_long_radix3_columns(E, op):
    """Column transforms of length 2025 = 3^4 5^2 (2005 rows, R = 20): more butterflies per
    pass than the component kernel takes with 4-column blocks, so it runs narrower blocks
    (a size the two-pass form refused before)."""
    c = E.Context(0)
    c.set_strategy(TWO_PASS)
    shape, S, K = (2005, 100), 41, 6
    assert c.fft_size(shape[0], (S - 1) // 2) == 2025
    img = blurred_noise(shape, 90)
    filt = random_filter(S, 91, 4.0 * S / 15)
    theta = theta_field(shape, 92)
    plan = E.FilterPlan.rotation(c, dev(filt), K)
    got = host(E.ecc_extended(c, op, plan, dev(img), dev(theta))).astype(np.float64)
    ref = oracle_corr(img, filt, theta, K, op)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    plan.close()
    c.close()


@pytest.mark.parametrize("shape", [(4096, 40), (40, 4096)], ids=["tall", "wide"])
@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_two_pass_transforms_above_4096(E, op, shape):
    """Two-pass transforms of 4116 points (4096 + R, 7-smooth): the plan's float64 filter
    spectra and the row kernels take 512-thread transforms there (refused before), except
    the correlation's combined inverse row kernel, which refuses rows that long."""
    c = E.Context(0)
    c.set_strategy(TWO_PASS)
    S, K = 21, 4
    assert c.fft_size(4096, (S - 1) // 2) == 4116
    img = blurred_noise(shape, 93)
    filt = random_filter(S, 94, 4.0 * S / 15)
    theta = theta_field(shape, 95)
    plan = E.FilterPlan.rotation(c, dev(filt), K)
    if op == 0 and shape[1] == 4096:
        with pytest.raises(E.EccError, match="too long"):
            E.ecc_extended(c, op, plan, dev(img), dev(theta))
        return
    got = host(E.ecc_extended(c, op, plan, dev(img), dev(theta))).astype(np.float64)
    ref = oracle_corr(img, filt, theta, K, op)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    plan.close()
    c.close()
