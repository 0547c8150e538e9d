"""GPU parity for rotation matching, scale-group smoothing and the convolution adjoint."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, random_filter, scale_field, theta_field, matching_scene

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


@pytest.fixture(scope="module")
def ctx(E):
    c = E.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------- matching

def check_matching(score, index, ref_score, C):
    assert relinf(score, ref_score) <= TOL and rel2(score, ref_score) <= TOL
    # index: unique where the best angle wins by a margin; otherwise it must attain the max
    srt = np.sort(C, axis=0)
    margin = (srt[-1] - srt[-2]) > 1e-4 * np.max(np.abs(C))
    ref_idx = np.argmax(C, axis=0)
    assert np.array_equal(index[margin], ref_idx[margin])
    picked = np.take_along_axis(C, index[None].astype(np.int64), axis=0)[0]
    assert np.all(np.abs(picked - ref_score) <= 2 * TOL * np.max(np.abs(C)))


@pytest.mark.parametrize("shape,S,K,A", [((96, 80), 15, 7, 64), ((70, 131), 9, 4, 17), ((64, 64), 21, 10, 32)])
def test_matching_parity(E, ctx, shape, S, K, A):
    img = blurred_noise(shape, 3)
    filt = random_filter(S, 4, 4.0 * S / 15)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    score, index = E.ecc_match_rotations(ctx, plan, dev(img), A)
    comps, _ = O.angular_components(filt, K)
    ref, _, C = O.match_rotations(img.astype(np.float64), comps, A)
    check_matching(host(score).astype(np.float64), host(index), ref, C)


def test_matching_full_size_recovers_planted_patterns(E, ctx):
    """1024^2 scene with a 63x63 pattern pasted three times (K = 16, 64 angles): parity
    with the oracle, and the three strongest peaks sit at the planted positions."""
    img, pat, truth = matching_scene(1024, 63)
    K = 16
    plan = E.FilterPlan.rotation(ctx, dev(pat), K)
    score, index = E.ecc_match_rotations(ctx, plan, dev(img), 64)
    score = host(score).astype(np.float64)
    index = host(index)
    comps, _ = O.angular_components(pat, K)
    ref, _, C = O.match_rotations(img.astype(np.float64), comps, 64)
    check_matching(score, index, ref, C)
    s = score.copy()
    for (r, c, a) in truth:
        i, j = np.unravel_index(np.argmax(s), s.shape)
        hit = [t for t in truth if abs(t[0] - i) <= 2 and abs(t[1] - j) <= 2]
        assert hit, (i, j, truth)
        m = int(round(hit[0][2] / (2 * np.pi) * 64)) % 64
        assert min(abs(int(index[i, j]) - m), 64 - abs(int(index[i, j]) - m)) <= 1
        s[max(0, i - 40):i + 40, max(0, j - 40):j + 40] = -np.inf


def test_matching_rejects_too_few_angles(E, ctx):
    plan = E.FilterPlan.rotation(ctx, dev(random_filter(9, 1, 2.0)), 8)
    with pytest.raises(E.EccError):
        E.ecc_match_rotations(ctx, plan, dev(blurred_noise((32, 32), 1)), 16)


# ---------------------------------------------------------------- scale group

SMALLP = dict(sigma0=1.0, scale_min=1.0, scale_max=2.0, components=12, period_factor=1.5)


def test_scale_components_match_oracle(E, ctx):
    plan = E.FilterPlan.scale(ctx, **SMALLP)
    p = O.ScaleParams(1.0, 1.0, 2.0, 12, 1.5)
    comps, w, om1 = O.scale_components(p)
    got = host(plan.components()).astype(np.complex128)
    assert got.shape == comps.shape
    assert np.max(np.abs(got - comps)) <= 2e-7 * np.max(np.abs(comps))


@pytest.mark.parametrize("shape", [(64, 80), (41, 57)])
def test_scale_smooth_parity(E, ctx, shape):
    plan = E.FilterPlan.scale(ctx, **SMALLP)
    img = blurred_noise(shape, 30)
    s = scale_field(shape, 31, 1.0, 2.0, sigma=4.0)
    y = host(E.ecc_scale_smooth(ctx, plan, dev(img), dev(s))).astype(np.float64)
    p = O.ScaleParams(1.0, 1.0, 2.0, 12, 1.5)
    ref, num, den = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), p)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


def test_scale_smooth_preserves_constants(E, ctx):
    plan = E.FilterPlan.scale(ctx, **SMALLP)
    s = scale_field((50, 60), 32, 1.0, 2.0, sigma=3.0)
    y = host(E.ecc_scale_smooth(ctx, plan, dev(np.full((50, 60), 0.37, np.float32)), dev(s)))
    assert np.max(np.abs(y - 0.37)) <= 1e-5


def test_scale_extended_convolution_parity(E, ctx):
    """Raw {H, s} * F (no normalisation) through ecc_extended with a scale plan."""
    plan = E.FilterPlan.scale(ctx, **SMALLP)
    img = blurred_noise((48, 52), 33)
    s = scale_field((48, 52), 34, 1.0, 2.0, sigma=3.0)
    y = host(E.ecc_extended(ctx, E.CONVOLUTION, plan, dev(img), dev(s))).astype(np.float64)
    p = O.ScaleParams(1.0, 1.0, 2.0, 12, 1.5)
    comps, w, om1 = O.scale_components(p)
    ref = O.ext_conv_half(img.astype(np.float64), om1 * np.log(s.astype(np.float64)), comps, w)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL


def test_scale_full_size_parity(E, ctx):
    """2048^2 scale-adaptive smoothing, 24 components, s in [1, 8]."""
    from synthetic import scale_config
    img, s = scale_config(2048)
    plan = E.FilterPlan.scale(ctx)
    y = host(E.ecc_scale_smooth(ctx, plan, dev(img), dev(s))).astype(np.float64)
    ref, _, _ = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), O.ScaleParams())
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("from_components", [False, True])
def test_convolution_adjoint_parity(E, ctx, from_components):
    import torch
    B, n, S, K = 3, 64, 11, 5
    imgs = np.stack([blurred_noise((n, n), 60 + i) for i in range(B)])
    ths = np.stack([theta_field((n, n), 70 + i) for i in range(B)])
    filt = random_filter(S, 80, 3.0)
    g = np.random.default_rng(81).standard_normal((B, n, n)).astype(np.float32)
    comps, _ = O.angular_components(filt, K)
    half = O.half_components(comps)
    if from_components:
        plan = E.FilterPlan.from_components(ctx, torch.from_numpy(half.astype(np.complex64)).cuda())
        half = half.astype(np.complex64).astype(np.complex128)
    else:
        plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    gs, gc, gf = E.ecc_extended_backward(ctx, plan, dev(imgs), dev(ths), dev(g))
    gs, gc, gf = host(gs).astype(np.float64), host(gc).astype(np.complex128), host(gf).astype(np.float64)
    rgc = np.zeros_like(half)
    for b in range(B):
        rh, rt, rc = O.conv_backward(imgs[b].astype(np.float64), ths[b].astype(np.float64), half,
                                     g[b].astype(np.float64))
        assert rel2(gs[b], rh) <= TOL and relinf(gs[b], rh) <= 2 * TOL
        assert rel2(gf[b], rt) <= TOL and relinf(gf[b], rt) <= 2 * TOL
        rgc += rc
    assert rel2(gc, rgc) <= TOL


@pytest.mark.parametrize("case", ["two_pass_strategy", "radius_without_block"])
def test_saved_stack_branch_matches_oracle(E, case):
    """The backward branch that reads a saved stack: the filter gradient of the two-pass
    form, reached with the two-pass strategy forced and, under the default strategy, with
    a radius no block shape covers (R = 57 > 56). Saved and recomputed stacks both match
    the float64 oracle gradient."""
    import torch
    if case == "two_pass_strategy":
        B, n, S, K = 2, 48, 9, 4
    else:
        B, n, S, K = 1, 120, 115, 3
    imgs = np.stack([blurred_noise((n, n), 90 + i) for i in range(B)])
    ths = np.stack([theta_field((n, n), 95 + i) for i in range(B)])
    g = np.random.default_rng(99).standard_normal((B, n, n)).astype(np.float32)
    filt = random_filter(S, 98, 2.5 * S / 9)
    c = E.Context(0)
    try:
        if case == "two_pass_strategy":
            c.set_strategy(E.STRATEGY_TWO_PASS)
        plan = E.FilterPlan.rotation(c, dev(filt), K)
        nbytes = E.ecc_backward_saved_size(c, plan, B, n, n)
        assert nbytes == B * (K + 1) * n * c.fft_size(n, (S - 1) // 2) * 8
        saved = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        y1 = host(E.ecc_extended_save(c, plan, dev(imgs), dev(ths), saved)).astype(np.float64)
        half = O.half_components(O.angular_components(filt, K)[0])
        grads = [E.ecc_extended_backward(c, plan, dev(imgs), dev(ths), dev(g), saved=sv)
                 for sv in (saved, None)]
        grads = [tuple(host(x) for x in gr) for gr in grads]
        plan.close()
    finally:
        c.close()
    rgc = np.zeros_like(half)
    for b in range(B):
        ref_y = O.ext_conv_half(imgs[b].astype(np.float64), ths[b].astype(np.float64), half)
        assert rel2(y1[b], ref_y) <= TOL
        rh, rt, rc = O.conv_backward(imgs[b].astype(np.float64), ths[b].astype(np.float64), half,
                                     g[b].astype(np.float64))
        for gs, gc, gf in grads:
            assert rel2(gs[b].astype(np.float64), rh) <= TOL
            assert rel2(gf[b].astype(np.float64), rt) <= TOL
        rgc += rc
    for gs, gc, gf in grads:
        assert rel2(gc.astype(np.complex128), rgc) <= TOL, rel2(gc.astype(np.complex128), rgc)


@pytest.mark.parametrize("checkpoint", [False, True])
def test_adjoint_full_size_through_autograd(E, ctx, checkpoint):
    """The differentiation workload at its real shape: 16 images of 512^2, a shared 21x21
    filter, K = 12, through the autograd function with a plan built from components (the
    general, non-symmetric block forms of the forward convolution, the signal/field
    correlation and the per-block filter lags). Every gradient against the float64
    oracle's at rel-L2 <= 1e-5: signal and field on four images, the components summed
    over all sixteen."""
    import torch
    from synthetic import adjoint_config
    imgs, thetas, filt, gbar = adjoint_config()
    B, K = imgs.shape[0], 12
    half = O.half_components(O.angular_components(filt, K)[0]).astype(np.complex64)
    H = dev(imgs).requires_grad_(True)
    T = dev(thetas).requires_grad_(True)
    Cc = torch.from_numpy(half).cuda().requires_grad_(True)
    y = E.ExtConv.apply(H, T, Cc, ctx, checkpoint)
    gi, gt, gc = torch.autograd.grad(y, (H, T, Cc), dev(gbar))
    y, gi, gt, gc = host(y), host(gi), host(gt), host(gc).astype(np.complex128)
    half64 = half.astype(np.complex128)
    rgc = np.zeros_like(half64)
    for b in range(B):
        img, th, gb = (a[b].astype(np.float64) for a in (imgs, thetas, gbar))
        rh, rt, rc = O.conv_backward(img, th, half64, gb)
        rgc += rc
        if b in (0, 5, 10, 15):
            ref_y = O.ext_conv_half(img, th, half64)
            assert rel2(y[b].astype(np.float64), ref_y) <= TOL
            assert rel2(gi[b].astype(np.float64), rh) <= TOL, (b, rel2(gi[b].astype(np.float64), rh))
            assert rel2(gt[b].astype(np.float64), rt) <= TOL, (b, rel2(gt[b].astype(np.float64), rt))
    assert rel2(gc, rgc) <= TOL, rel2(gc, rgc)


def test_autograd_function(E, ctx):
    import torch
    n, S, K = 40, 9, 4
    img = torch.from_numpy(blurred_noise((n, n), 7)).cuda().requires_grad_(True)
    th = torch.from_numpy(theta_field((n, n), 8)).cuda().requires_grad_(True)
    comps, _ = O.angular_components(random_filter(S, 9, 2.5), K)
    half = torch.from_numpy(O.half_components(comps).astype(np.complex64)).cuda().requires_grad_(True)
    for ckpt in (False, True):
        y = E.ExtConv.apply(img, th, half, ctx, ckpt)
        gy = torch.randn_like(y)
        gi, gt, gc = torch.autograd.grad(y, (img, th, half), gy)
        rh, rt, rc = O.conv_backward(img.detach().cpu().numpy().astype(np.float64),
                                     th.detach().cpu().numpy().astype(np.float64),
                                     half.detach().cpu().numpy().astype(np.complex128),
                                     gy.cpu().numpy().astype(np.float64))
        assert rel2(gi.cpu().numpy().astype(np.float64), rh) <= TOL
        assert rel2(gt.cpu().numpy().astype(np.float64), rt) <= TOL
        assert rel2(gc.cpu().numpy().astype(np.complex128), rc) <= TOL


@pytest.mark.parametrize("strategy", ["auto", "two_pass"])
@pytest.mark.parametrize("from_components", [False, True])
def test_correlation_adjoint_parity(E, from_components, strategy):
    """Adjoint of the extended correlation (signal, angle field and components) against
    the oracle's gradients, with the block strategy (N = 64 blocks) and the two-pass one."""
    import torch
    B, n, S, K = 2, 64, 11, 5
    imgs = np.stack([blurred_noise((n, n), 160 + i) for i in range(B)])
    ths = np.stack([theta_field((n, n), 170 + i) for i in range(B)])
    filt = random_filter(S, 180, 3.0)
    g = np.random.default_rng(181).standard_normal((B, n, n)).astype(np.float32)
    comps, _ = O.angular_components(filt, K)
    half = O.half_components(comps)
    c = E.Context(0)
    try:
        if strategy == "two_pass":
            c.set_strategy(E.STRATEGY_TWO_PASS)
        if from_components:
            plan = E.FilterPlan.from_components(c, torch.from_numpy(half.astype(np.complex64)).cuda())
            half = half.astype(np.complex64).astype(np.complex128)
        else:
            plan = E.FilterPlan.rotation(c, dev(filt), K)
        gs, gc, gf = E.ecc_extended_backward(c, plan, dev(imgs), dev(ths), dev(g), op=E.CORRELATION)
        gs, gc, gf = host(gs).astype(np.float64), host(gc).astype(np.complex128), host(gf).astype(np.float64)
        plan.close()
    finally:
        c.close()
    rgc = np.zeros_like(half)
    for b in range(B):
        rh, rt, rc = O.corr_backward(imgs[b].astype(np.float64), ths[b].astype(np.float64), half,
                                     g[b].astype(np.float64))
        assert rel2(gs[b], rh) <= TOL and relinf(gs[b], rh) <= 2 * TOL
        assert rel2(gf[b], rt) <= TOL and relinf(gf[b], rt) <= 2 * TOL
        rgc += rc
    assert rel2(gc, rgc) <= TOL


def test_correlation_adjoint_symmetric_pair_form(E):
    """The field part through the symmetric N = 96 pair form (a large image, radius 15)."""
    S, K = 31, 6
    filt = random_filter(S, 192, 4.0 * S / 15)
    c = E.Context(0)
    try:
        plan = E.FilterPlan.rotation(c, dev(filt), K)
        shapes = [sh for sh in ((520, 491), (700, 653), (1024, 1000))
                  if c.describe(E.CORRELATION, plan, *sh)[:2] == (E.STRATEGY_TILED, 96)]
        assert shapes, "no candidate shape runs N = 96 blocks"
        shape = shapes[0]
        img = blurred_noise(shape, 190)
        th = theta_field(shape, 191)
        g = np.random.default_rng(193).standard_normal(shape).astype(np.float32)
        gs, gc, gf = E.ecc_extended_backward(c, plan, dev(img), dev(th), dev(g), op=E.CORRELATION)
        gs, gc, gf = host(gs).astype(np.float64), host(gc).astype(np.complex128), host(gf).astype(np.float64)
        plan.close()
    finally:
        c.close()
    comps, _ = O.angular_components(filt, K)
    rh, rt, rc = O.corr_backward(img.astype(np.float64), th.astype(np.float64), O.half_components(comps),
                                 g.astype(np.float64))
    assert rel2(gs, rh) <= TOL and relinf(gs, rh) <= 2 * TOL
    assert rel2(gf, rt) <= TOL and relinf(gf, rt) <= 2 * TOL
    assert rel2(gc, rc) <= TOL


def test_correlation_adjoint_rejects_saved_stack(E, ctx):
    import torch
    plan = E.FilterPlan.rotation(ctx, dev(random_filter(9, 194, 2.5)), 3)
    x = dev(blurred_noise((32, 32), 195))
    saved = torch.empty(16, dtype=torch.float32, device="cuda")
    with pytest.raises(E.EccError):
        E.ecc_extended_backward(ctx, plan, x, x.clone(), x.clone(), saved=saved, op=E.CORRELATION)


def test_autograd_correlation_function(E, ctx):
    import torch
    n, S, K = 40, 9, 4
    img = torch.from_numpy(blurred_noise((n, n), 17)).cuda().requires_grad_(True)
    th = torch.from_numpy(theta_field((n, n), 18)).cuda().requires_grad_(True)
    comps, _ = O.angular_components(random_filter(S, 19, 2.5), K)
    half = torch.from_numpy(O.half_components(comps).astype(np.complex64)).cuda().requires_grad_(True)
    y = E.ExtCorr.apply(img, th, half, ctx)
    gy = torch.randn_like(y)
    gi, gt, gc = torch.autograd.grad(y, (img, th, half), gy)
    rh, rt, rc = O.corr_backward(img.detach().cpu().numpy().astype(np.float64),
                                 th.detach().cpu().numpy().astype(np.float64),
                                 half.detach().cpu().numpy().astype(np.complex128),
                                 gy.cpu().numpy().astype(np.float64))
    assert rel2(gi.cpu().numpy().astype(np.float64), rh) <= TOL
    assert rel2(gt.cpu().numpy().astype(np.float64), rt) <= TOL
    assert rel2(gc.cpu().numpy().astype(np.complex128), rc) <= TOL
