"""Context workspace sizing (ecc_workspace_size / _reserve / _allocated).

For every call that uses the context workspace, on a fresh context: the size reported
before the call equals what the call then allocates (the workspace grows to exactly what
a call needs), and after reserving that size the call allocates nothing more. Outputs of
the reserved run are checked against the float64 oracle so the sizes are not met by a
path that skipped work."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, random_filter, scale_field, theta_field

pytestmark = pytest.mark.gpu
TOL = 1e-5


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def E():
    import torch
    import paper_2006_13188_amd as E_
    assert torch.cuda.is_available()
    E_.lib()
    return E_


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rotation_case(shape, S, K, seed):
    img = blurred_noise(shape, seed)
    th = theta_field(shape, seed + 1)
    filt = random_filter(S, seed + 2, 4.0 * S / 15)
    half = O.half_components(O.angular_components(filt, K)[0])
    return img, th, filt, half


def run_call(E, c, call, plan, img, th):
    """Runs `call` once; returns (output arrays, oracle values)."""
    if call in (E.WS_EXTENDED_CORRELATION, E.WS_EXTENDED_CONVOLUTION):
        return host(E.ecc_extended(c, call, plan, dev(img), dev(th)))
    if call == E.WS_MATCH_ROTATIONS:
        score, _ = E.ecc_match_rotations(c, plan, dev(img), 32)
        return host(score)
    if call == E.WS_SCALE_SMOOTH:
        return host(E.ecc_scale_smooth(c, plan, dev(img), dev(th)))
    op = E.CONVOLUTION if call == E.WS_BACKWARD_CONVOLUTION else E.CORRELATION
    g = np.random.default_rng(5).standard_normal(img.shape).astype(np.float32)
    gs, gc, gf = E.ecc_extended_backward(c, plan, dev(img[None]), dev(th[None]), dev(g[None]), op=op)
    return host(gs)[0]


def reference(E, call, img, th, half):
    a, t = img.astype(np.float64), th.astype(np.float64)
    if call == E.WS_EXTENDED_CORRELATION:
        return O.ext_corr_half(a, t, half)
    if call == E.WS_EXTENDED_CONVOLUTION:
        return O.ext_conv_half(a, t, half)
    if call == E.WS_MATCH_ROTATIONS:
        return O.match_rotations(a, np.concatenate([np.conj(half[:0:-1]), half]), 32)[0]
    g = np.random.default_rng(5).standard_normal(img.shape).astype(np.float32).astype(np.float64)
    if call == E.WS_BACKWARD_CONVOLUTION:
        return O.conv_backward(a, t, half, g)[0]
    return O.corr_backward(a, t, half, g)[0]


CASES = [
    ("corr", "tiled", ((150, 131), 15, 6)),
    ("corr", "two_pass", ((150, 131), 15, 6)),
    ("conv", "tiled", ((150, 131), 15, 6)),
    ("conv", "two_pass", ((150, 131), 15, 6)),
    ("match", "tiled", ((150, 131), 15, 6)),
    ("match", "two_pass", ((150, 131), 15, 6)),
    ("bconv", "tiled", ((150, 131), 15, 6)),
    ("bconv", "two_pass", ((150, 131), 15, 6)),
    ("bcorr", "tiled", ((150, 131), 15, 6)),
    ("bcorr", "two_pass", ((150, 131), 15, 6)),
]


@pytest.mark.parametrize("what,strategy,shape_s_k", CASES,
                         ids=[f"{a}-{b}" for a, b, _ in CASES])
@pytest.mark.parametrize("reserve", [False, True], ids=["grow", "reserved"])
def test_reported_size_is_what_the_call_uses(E, what, strategy, shape_s_k, reserve):
    calls = {"corr": E.WS_EXTENDED_CORRELATION, "conv": E.WS_EXTENDED_CONVOLUTION,
             "match": E.WS_MATCH_ROTATIONS, "bconv": E.WS_BACKWARD_CONVOLUTION,
             "bcorr": E.WS_BACKWARD_CORRELATION}
    call = calls[what]
    shape, S, K = shape_s_k
    img, th, filt, half = rotation_case(shape, S, K, 300)
    c = E.Context(0)
    try:
        c.set_strategy(E.STRATEGY_TILED if strategy == "tiled" else E.STRATEGY_TWO_PASS)
        plan = E.FilterPlan.rotation(c, dev(filt), K)
        need = c.workspace_size(call, plan, *shape)
        if strategy == "tiled" and what in ("corr", "conv"):
            assert need == 0
        if strategy == "two_pass" or what == "match":
            assert need > 0
        if reserve:
            c.workspace_reserve(need)
            assert c.workspace_allocated() == need
        y = run_call(E, c, call, plan, img, th)
        assert c.workspace_allocated() == need
        # a second call of the same shape allocates nothing either
        run_call(E, c, call, plan, img, th)
        assert c.workspace_allocated() == need
        plan.close()
    finally:
        c.close()
    ref = reference(E, call, img, th, half)
    assert rel2(y.astype(np.float64), ref) <= TOL


@pytest.mark.parametrize("strategy", ["auto", "tiled", "two_pass"])
def test_scale_smoothing_workspace(E, strategy):
    shape = (150, 170)
    img = blurred_noise(shape, 320)
    s = scale_field(shape, 321)
    c = E.Context(0)
    try:
        c.set_strategy({"auto": E.STRATEGY_AUTO, "tiled": E.STRATEGY_TILED, "two_pass": E.STRATEGY_TWO_PASS}[strategy])
        plan = E.FilterPlan.scale(c)
        need = c.workspace_size(E.WS_SCALE_SMOOTH, plan, *shape)
        assert need == c.workspace_size(E.WS_NORMALIZED_CONVOLUTION, plan, *shape)
        if strategy == "auto":
            # radius 32: 128-point blocks, the overlap-add ratio kernel: 3 x 3 blocks of
            # 64 x 64 sources, a 128 x 128 complex64 region each
            assert need == 9 * 128 * 128 * 8
        elif strategy == "tiled":
            # any block side >= 16 allowed: 96-point blocks of 32 x 32 (two launches, no
            # workspace) cost less for so small an image
            assert need == 0
        y = host(E.ecc_scale_smooth(c, plan, dev(img), dev(s)))
        assert c.workspace_allocated() == need
        plan.close()
    finally:
        c.close()
    ref = O.scale_smooth_fft(img.astype(np.float64), s.astype(np.float64), O.ScaleParams())[0]
    assert rel2(y.astype(np.float64), ref) <= TOL


def test_workspace_query_rejects_bad_arguments(E):
    c = E.Context(0)
    try:
        plan = E.FilterPlan.rotation(c, dev(random_filter(9, 7, 2.5)), 3)
        with pytest.raises(E.EccError):
            c.workspace_size(99, plan, 64, 64)
        with pytest.raises(E.EccError):
            c.workspace_size(E.WS_EXTENDED_CORRELATION, plan, 0, 64)
        with pytest.raises(E.EccError):
            c.workspace_size(E.WS_SCALE_SMOOTH, plan, 64, 64)   # needs a scale plan
        plan.close()
    finally:
        c.close()
