"""Rotation-invariant matching: both strategies and the three angle-search precisions
against the float64 oracle.

Tolerances (score, rel-inf and rel-L2 against the oracle): float32 1e-5; float16 hi/lo
matrix cores 1e-5 (hi + lo keeps ~22 bits per operand, the dropped lo*lo term is
~2^-22 relative); bfloat16 hi/lo 1e-4 (8 + 8 bits, ~2^-16 relative per product). The
index is compared where the best angle wins by more than the precision's error margin,
and must otherwise attain the maximum within tolerance."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, matching_scene, random_filter

pytestmark = pytest.mark.gpu
TWO_PASS, TILED = 1, 2
FP32, FP16_HILO, BF16_HILO = 0, 1, 2
TOLS = {FP32: 1e-5, FP16_HILO: 1e-5, BF16_HILO: 1e-4}


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


def check(score, index, ref, C, tol):
    assert relinf(score, ref) <= tol and rel2(score, ref) <= tol, (relinf(score, ref), rel2(score, ref))
    srt = np.sort(C, axis=0)
    scale = np.max(np.abs(C))
    margin = (srt[-1] - srt[-2]) > 10 * tol * scale
    assert np.array_equal(index[margin], np.argmax(C, axis=0)[margin])
    picked = np.take_along_axis(C, index[None].astype(np.int64), axis=0)[0]
    assert np.all(np.abs(picked - ref) <= 2 * tol * scale)


@pytest.mark.parametrize("prec", [FP32, FP16_HILO, BF16_HILO], ids=["fp32", "fp16_hilo", "bf16_hilo"])
@pytest.mark.parametrize("shape,S,K,A", [((96, 80), 15, 7, 64), ((70, 131), 9, 4, 17), ((64, 64), 21, 10, 32),
                                         ((150, 140), 63, 16, 64), ((40, 200), 7, 31, 63), ((60, 90), 11, 23, 64),
                                         ((48, 72), 9, 31, 64)])
def test_matching_parity(E, sctx, prec, shape, S, K, A):
    ctx, strat = sctx
    img = blurred_noise(shape, 3)
    filt = random_filter(S, 4, 4.0 * S / 15)
    plan = E.FilterPlan.rotation(ctx, dev(filt), K)
    if strat == TWO_PASS and prec != FP32:
        with pytest.raises(E.EccError):
            E.ecc_match_rotations(ctx, plan, dev(img), A, precision=prec)
        return
    score, index = E.ecc_match_rotations(ctx, plan, dev(img), A, precision=prec)
    comps, _ = O.angular_components(filt, K)
    ref, _, C = O.match_rotations(img.astype(np.float64), comps, A)
    check(host(score).astype(np.float64), host(index), ref, C, TOLS[prec])


@pytest.mark.parametrize("prec", [FP32, FP16_HILO, BF16_HILO], ids=["fp32", "fp16_hilo", "bf16_hilo"])
def test_full_size_planted_patterns(E, prec):
    """1024^2 scene, 63x63 pattern pasted three times, K = 16, 64 angles (default
    strategy): parity with the oracle and the planted positions and angles recovered."""
    img, pat, truth = matching_scene(1024, 63)
    ctx = E.Context(0)
    try:
        plan = E.FilterPlan.rotation(ctx, dev(pat), 16)
        score, index = E.ecc_match_rotations(ctx, plan, dev(img), 64, precision=prec)
        score = host(score).astype(np.float64)
        index = host(index)
    finally:
        ctx.close()
    comps, _ = O.angular_components(pat, 16)
    ref, _, C = O.match_rotations(img.astype(np.float64), comps, 64)
    check(score, index, ref, C, TOLS[prec])
    s = score.copy()
    for _ in truth:
        i, j = np.unravel_index(np.argmax(s), s.shape)
        hit = [t for t in truth if abs(t[0] - i) <= 2 and abs(t[1] - j) <= 2]
        assert hit, (i, j, truth)
        m = int(round(hit[0][2] / (2 * np.pi) * 64)) % 64
        assert min(abs(int(index[i, j]) - m), 64 - abs(int(index[i, j]) - m)) <= 1
        s[max(0, i - 40):i + 40, max(0, j - 40):j + 40] = -np.inf


@pytest.mark.parametrize("shape,A", [((40, 2600), 16), ((30, 1025), 64)])
def test_two_pass_matching_wide_rows(E, shape, A):
    """Two-pass matching of rows wider than one workgroup's 1024 pixels: the rows are split
    into segments, each transforming the whole row (was refused)."""
    c = E.Context(0)
    c.set_strategy(TWO_PASS)
    img = blurred_noise(shape, 5)
    S, K = 21, 6
    filt = random_filter(S, 6, 4.0 * S / 15)
    plan = E.FilterPlan.rotation(c, dev(filt), K)
    score, index = E.ecc_match_rotations(c, plan, dev(img), A)
    comps, _ = O.angular_components(filt, K)
    ref, _, C = O.match_rotations(img.astype(np.float64), comps, A)
    check(host(score).astype(np.float64), host(index), ref, C, TOLS[FP32])
    plan.close()
    c.close()
