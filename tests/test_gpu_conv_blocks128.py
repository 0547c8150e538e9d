"""The extended convolution by 128-point overlap-add blocks (filter radii 25..32 under the
default strategy), against the float64 oracle: ragged image sizes (partial blocks, images
smaller than a block), batches, odd and even band limits, the largest radius, a scale plan,
and the workspace query. Tolerance: rel-L2 and rel-inf <= 1e-5."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, random_filter, scale_field, theta_field

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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape,S,K,batch", [((150, 211), 53, 6, 1), ((64, 300), 51, 5, 2), ((97, 97), 63, 16, 1),
                                             ((200, 130), 65, 3, 1), ((60, 70), 57, 0, 1)])
def test_overlap_add_convolution_matches_the_oracle(E, ctx, shape, S, K, batch):
    imgs = np.stack([blurred_noise(shape, 100 + S + b) for b in range(batch)])
    ths = np.stack([theta_field(shape, 200 + S + b) for b in range(batch)])
    filt = random_filter(S, 300 + K, 4.0 * S / 15)
    print(f"overlap-add conv shape={shape} S={S} K={K} batch={batch}", flush=True)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    assert ctx.describe(E.CONVOLUTION, plan, *shape)[:2] == (E.STRATEGY_TILED, 128)
    n = ctx.workspace_size(E.WS_EXTENDED_CONVOLUTION, plan, *shape, batch=batch)
    assert n > 0
    got = host(E.ecc_extended(ctx, E.CONVOLUTION, plan, dev(imgs if batch > 1 else imgs[0]),
                              dev(ths if batch > 1 else ths[0])))
    got = got.reshape((batch,) + shape)
    comps, _ = O.angular_components(filt, K)
    half = O.half_components(comps)
    for b in range(batch):
        ref = O.ext_conv_half(imgs[b].astype(np.float64), ths[b].astype(np.float64), half)
        assert rel2(got[b], ref) <= TOL and relinf(got[b], ref) <= TOL, (b, rel2(got[b], ref), relinf(got[b], ref))
    again = host(E.ecc_extended(ctx, E.CONVOLUTION, plan, dev(imgs if batch > 1 else imgs[0]),
                                dev(ths if batch > 1 else ths[0]))).reshape((batch,) + shape)
    assert np.array_equal(got, again)
    plan.close()


def test_overlap_add_convolution_scale_plan(E, ctx):
    """A scale plan whose support takes 128-point blocks: field = scale, phase omega_1 ln s."""
    plan = E.FilterPlan.scale(ctx, sigma0=3.5, scale_min=1.0, scale_max=2.0, components=9)
    p = O.ScaleParams(3.5, 1.0, 2.0, 9, 1.5)
    assert 25 <= p.R <= 32
    comps, w, om1 = O.scale_components(p)
    shape = (120, 170)
    assert ctx.describe(E.CONVOLUTION, plan, *shape)[:2] == (E.STRATEGY_TILED, 128)
    img = blurred_noise(shape, 61)
    s = scale_field(shape, 62, 1.0, 2.0, sigma=4.0)
    got = host(E.ecc_extended(ctx, E.CONVOLUTION, plan, dev(img), dev(s)))
    ref = O.ext_conv_half(img.astype(np.float64), om1 * np.log(s.astype(np.float64)), comps, w)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    plan.close()
