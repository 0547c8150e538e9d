"""GPU parity of the HIP path against the float64 oracle (rotation group).

Tolerance (float32 path vs float64 oracle): rel-L2 <= 1e-5 and rel-inf <= 1e-5, where
rel-inf = max|y - y_ref| / max|y_ref|. Matching indices are compared where the best
angle wins by a margin (several angles are valid maxima otherwise)."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, random_filter, rotation_config, theta_field

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
    E_.lib()  # fails loudly if the library is missing
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
    return t.cpu().numpy()


def run(E, ctx, op, img, filt, theta, K):
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    y = E.ecc_extended(ctx, op, plan, dev(img), dev(theta))
    return host(y).astype(np.float64), plan


def oracle_out(op, img, filt, theta, K):
    comps, _ = O.angular_components(filt, K)
    half = O.half_components(comps)
    f = O.ext_corr_half if op == 0 else O.ext_conv_half
    return f(img.astype(np.float64), theta.astype(np.float64), half)


def test_components_match_oracle(E, ctx):
    img, filt, theta, K = rotation_config(128, 15, 8)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    assert (plan.S, plan.K, plan.M) == (15, 8, 256)
    got = host(plan.components()).astype(np.complex128)
    comps, _ = O.angular_components(filt, K)
    ref = O.half_components(comps)
    assert np.max(np.abs(got - ref)) <= 2e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("op", [0, 1])
def test_small_config_parity(E, ctx, op):
    img, filt, theta, K = rotation_config(128, 15, 8)
    y, _ = run(E, ctx, op, img, filt, theta, K)
    ref = oracle_out(op, img, filt, theta, K)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


@pytest.mark.parametrize("shape,S,K", [((67, 93), 9, 3), ((130, 41), 7, 2), ((33, 33), 31, 12),
                                       ((200, 173), 21, 10)])
@pytest.mark.parametrize("op", [0, 1])
def test_ragged_shapes_parity(E, ctx, op, shape, S, K):
    img = blurred_noise(shape, 5)
    filt = random_filter(S, 6, 4.0 * S / 15)
    theta = theta_field(shape, 7)
    y, _ = run(E, ctx, op, img, filt, theta, K)
    ref = oracle_out(op, img, filt, theta, K)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


@pytest.mark.parametrize("op", [0, 1])
def test_batch_matches_single_images(E, ctx, op):
    import torch
    imgs = np.stack([blurred_noise((70, 64), 40 + i) for i in range(3)])
    ths = np.stack([theta_field((70, 64), 50 + i) for i in range(3)])
    filt = random_filter(11, 8, 3.0)
    plan = E.FilterPlan.rotation(ctx, dev(filt), 5)
    yb = host(E.ecc_extended(ctx, op, plan, dev(imgs), dev(ths)))
    for i in range(3):
        ref = oracle_out(op, imgs[i], filt, ths[i], 5)
        assert rel2(yb[i].astype(np.float64), ref) <= TOL


def test_radial_filter_ignores_field(E, ctx):
    img, filt, theta, _ = rotation_config(96, 13, 4)
    plan = E.FilterPlan.rotation(ctx, dev(filt), 0)
    a = host(E.ecc_extended(ctx, 0, plan, dev(img), dev(theta)))
    b = host(E.ecc_extended(ctx, 0, plan, dev(img), dev(np.zeros_like(theta))))
    assert np.array_equal(a, b)


def test_steerable_closed_form_on_gpu(E, ctx):
    """Components of d/dx of a Gaussian (k = +-1 only) steer as cos G_x + sin G_y."""
    import scipy.signal as ss
    S, sig = 13, 2.0
    R = 6
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    r = np.hypot(xx, yy)
    disk = r <= R
    g = np.exp(-r ** 2 / (2 * sig ** 2))
    comps = np.zeros((2, S, S), np.complex64)
    comps[1] = np.where(disk, -(r * g) / (2 * sig ** 2) * np.exp(1j * np.arctan2(yy, xx)), 0)
    import torch
    plan = E.FilterPlan.from_components(ctx, torch.from_numpy(comps).cuda())
    img = blurred_noise((90, 77), 3)
    th = theta_field((90, 77), 4)
    y = host(E.ecc_extended(ctx, 0, plan, dev(img), dev(th))).astype(np.float64)
    Gx = np.where(disk, -xx / sig ** 2 * g, 0)
    Gy = np.where(disk, -yy / sig ** 2 * g, 0)
    H = img.astype(np.float64)
    t = th.astype(np.float64)
    ref = np.cos(t) * ss.correlate2d(H, Gx, mode="same") + np.sin(t) * ss.correlate2d(H, Gy, mode="same")
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL


@pytest.mark.parametrize("op", [0, 1])
def test_full_size_parity(E, ctx, op):
    """1024 x 1024 image, 31 x 31 filter, K = 16, against the float64 FFT oracle."""
    img, filt, theta, K = rotation_config(1024, 31, 16, seeds=(10, 11, 12))
    y, _ = run(E, ctx, op, img, filt, theta, K)
    ref = oracle_out(op, img, filt, theta, K)
    assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (rel2(y, ref), relinf(y, ref))


def test_full_size_sampled_brute_force(E, ctx):
    """Sampled pixels of the 1024^2 correlation against the definition, one by one."""
    img, filt, theta, K = rotation_config(1024, 31, 16, seeds=(10, 11, 12))
    y, _ = run(E, ctx, 0, img, filt, theta, K)
    comps, _ = O.angular_components(filt, K)
    rng = np.random.default_rng(0)
    pts = [(0, 0), (1023, 1023), (0, 1023), (7, 512)] + [tuple(rng.integers(0, 1024, 2)) for _ in range(40)]
    H = img.astype(np.float64)
    R = 15
    Hp = np.pad(H, R)
    scale = np.max(np.abs(y))
    for (i, j) in pts:
        Ft = O.rotated_filter(comps, float(theta[i, j]))
        ref = np.sum(Hp[i:i + 31, j:j + 31] * np.conj(Ft)).real
        assert abs(y[i, j] - ref) <= TOL * scale


def test_invalid_arguments(E, ctx):
    import torch
    filt = random_filter(15, 1, 4.0)
    with pytest.raises(E.EccError):
        E.FilterPlan.rotation(ctx, dev(np.zeros((14, 14), np.float32)), 3)   # even side
    with pytest.raises(E.EccError):
        E.FilterPlan.rotation(ctx, dev(filt), 200)                            # K > M/2 - 1
    plan = E.FilterPlan.rotation(ctx, dev(filt), 4)
    small = dev(np.zeros((10, 10), np.float32))
    with pytest.raises(E.EccError):
        E.ecc_extended(ctx, 0, plan, small, small)                            # filter > image
    img = dev(blurred_noise((64, 64), 1))
    with pytest.raises(E.EccError):
        E.ecc_extended(ctx, 0, plan, img, img, out=img)                       # aliasing
    out = torch.full((64, 64), 7.0, device="cuda")
    with pytest.raises(E.EccError):
        E.ecc_extended(ctx, 2, plan, img, img, out=out)                       # bad op
    assert torch.all(out == 7.0)                                               # untouched


def test_repeatable(E, ctx):
    img, filt, theta, K = rotation_config(256, 21, 10)
    a, plan = run(E, ctx, 0, img, filt, theta, K)
    b = host(E.ecc_extended(ctx, 0, plan, dev(img), dev(theta)))
    assert np.array_equal(a.astype(np.float32), b)
