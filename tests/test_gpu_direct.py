"""The direct (spatial) extended correlation and convolution for small filters, against
the float64 oracle: every compiled filter side (3..15) with several band limits, on ragged
image shapes that cover partial 16 x 64 blocks and images smaller than a block, batches, a
scale-group plan (logarithmic field) and components given directly; the strategy query,
the workspace query and the errors. Tolerance: rel-L2 and rel-inf <= 1e-5."""
import numpy as np
import pytest

import oracle as O
from synthetic import anisotropic_gaussian, blurred_noise, random_filter, scale_field, theta_field

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
def dctx(E):
    c = E.Context(0)
    c.set_strategy(E.STRATEGY_DIRECT)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_corr(img, filt, theta, K, op=0):
    comps, _ = O.angular_components(filt, K)
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    return f(img.astype(np.float64), theta.astype(np.float64), O.half_components(comps))


@pytest.mark.parametrize("shape,S,K", [
    ((37, 130), 3, 1), ((64, 64), 5, 2), ((100, 71), 7, 4), ((16, 64), 9, 3), ((129, 200), 11, 6),
    ((45, 45), 13, 8), ((90, 33), 15, 5), ((17, 65), 7, 0), ((15, 15), 15, 16), ((3, 5), 3, 1)])
@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_direct_matches_the_oracle(E, dctx, shape, S, K, op):
    img = blurred_noise(shape, 11 + S)
    filt = random_filter(S, 12 + K, 4.0 * S / 15)
    th = theta_field(shape, 13)
    print(f"direct op={op} shape={shape} S={S} K={K}", flush=True)
    plan = E.FilterPlan.rotation(dctx, dev(filt), K)
    assert dctx.describe(op, plan, *shape)[:2] == (E.STRATEGY_DIRECT, 0)
    ws = E.WS_EXTENDED_CORRELATION if op == 0 else E.WS_EXTENDED_CONVOLUTION
    assert dctx.workspace_size(ws, plan, *shape) == 0
    got = host(E.ecc_extended(dctx, op, plan, dev(img), dev(th)))
    ref = oracle_corr(img, filt, th, K, op)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    again = host(E.ecc_extended(dctx, op, plan, dev(img), dev(th)))
    assert np.array_equal(got, again)
    plan.close()


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_direct_batch(E, dctx, op):
    B, shape, S, K = 3, (70, 150), 9, 4
    imgs = np.stack([blurred_noise(shape, 20 + b) for b in range(B)])
    ths = np.stack([theta_field(shape, 25 + b) for b in range(B)])
    filt = random_filter(S, 30, 2.5)
    plan = E.FilterPlan.rotation(dctx, dev(filt), K)
    got = host(E.ecc_extended(dctx, op, plan, dev(imgs), dev(ths)))
    for b in range(B):
        ref = oracle_corr(imgs[b], filt, ths[b], K, op)
        assert rel2(got[b], ref) <= TOL and relinf(got[b], ref) <= TOL
    plan.close()


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_direct_scale_group(E, dctx, op):
    """A scale plan (log-radial components, field = scale, phase omega_1 ln s)."""
    plan = E.FilterPlan.scale(dctx, sigma0=0.8, scale_min=1.0, scale_max=1.5, components=12)
    p = O.ScaleParams(0.8, 1.0, 1.5, 12, 1.5)
    comps, w, om1 = O.scale_components(p)
    assert comps.shape[1] <= 15
    shape = (77, 91)
    img = blurred_noise(shape, 40)
    s = scale_field(shape, 41, 1.0, 1.5, sigma=4.0)
    assert dctx.describe(op, plan, *shape)[0] == E.STRATEGY_DIRECT
    got = host(E.ecc_extended(dctx, op, plan, dev(img), dev(s)))
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    ref = f(img.astype(np.float64), om1 * np.log(s.astype(np.float64)), comps, w)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    plan.close()


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_direct_from_components(E, dctx, op):
    """Components given directly (no parity assumed): the same sums."""
    import torch
    S, K, shape = 7, 3, (50, 61)
    filt = random_filter(S, 50, 2.0)
    comps, _ = O.angular_components(filt, K)
    half = O.half_components(comps)
    plan = E.FilterPlan.from_components(dctx, torch.from_numpy(half.astype(np.complex64)).cuda())
    img = blurred_noise(shape, 51)
    th = theta_field(shape, 52)
    got = host(E.ecc_extended(dctx, op, plan, dev(img), dev(th)))
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    ref = f(img.astype(np.float64), th.astype(np.float64), half)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL
    plan.close()


def test_direct_strategy_limits(E, dctx):
    """Filters above 15 are refused under DIRECT (both ops); calls other than ecc_extended
    (here the normalised convolution) run as under AUTO."""
    shape = (40, 48)
    big = E.FilterPlan.rotation(dctx, dev(random_filter(17, 60, 4.0)), 3)
    img, th = dev(blurred_noise(shape, 61)), dev(theta_field(shape, 62))
    for op in (E.CORRELATION, E.CONVOLUTION):
        with pytest.raises(E.EccError):
            E.ecc_extended(dctx, op, big, img, th)
    big.close()
    filt = anisotropic_gaussian(9, 2.0, 0.8)        # positive: a well-conditioned ratio
    plan = E.FilterPlan.rotation(dctx, dev(filt), 4)
    got = host(E.ecc_normalized_convolution(dctx, plan, img, th))
    comps, _ = O.angular_components(filt, 4)
    H = blurred_noise(shape, 61).astype(np.float64)
    a = theta_field(shape, 62).astype(np.float64)
    half = O.half_components(comps)
    ref = O.ext_conv_half(H, a, half) / O.ext_conv_half(np.ones_like(H), a, half)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL
    plan.close()


@pytest.mark.parametrize("op", [0, 1], ids=["corr", "conv"])
def test_auto_takes_the_direct_sums_for_the_smallest_filters(E, op):
    """AUTO compares the two forms' modelled times: 3 x 3 and 5 x 5 filters go direct at
    every band limit here, 11 x 11 and larger take blocks."""
    c = E.Context(0)
    shape = (512, 512)
    for S, K, want in ((3, 8, E.STRATEGY_DIRECT), (5, 16, E.STRATEGY_DIRECT), (11, 4, E.STRATEGY_TILED),
                       (15, 2, E.STRATEGY_TILED)):
        filt = random_filter(S, 70 + S, 4.0 * S / 15)
        plan = E.FilterPlan.rotation(c, dev(filt), K)
        assert c.describe(op, plan, *shape)[0] == want, (S, K)
        if S == 3:
            img, th = blurred_noise(shape, 71), theta_field(shape, 72)
            got = host(E.ecc_extended(c, op, plan, dev(img), dev(th)))
            ref = oracle_corr(img, filt, th, K, op)
            assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL
        plan.close()
    c.close()
