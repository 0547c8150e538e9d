"""Pattern detection (Sec. 5) on the GPU against the float64 oracle: the gradient signal and
field, the consensus filter by voting, peak picking (exact lists on the same response),
and the whole detection on the 1024 x 1024 scene of the matching workload (three rotated
63 x 63 patterns pasted into noise)."""
import numpy as np
import pytest

import oracle as O
from synthetic import blurred_noise, matching_scene, random_filter

pytestmark = pytest.mark.gpu


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


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


def check_field(H, th, img):
    rH, rth = O.gradient_field(img.astype(np.float64))
    assert rel2(H.astype(np.float64), rH) <= 1e-6
    ok = rH > 1e-4 * rH.max()        # the angle of a vanishing gradient is not defined
    d = np.angle(np.exp(1j * (th.astype(np.float64) - rth)))
    assert np.max(np.abs(d[ok])) <= 1e-5


@pytest.mark.parametrize("shape", [(97, 130), (2, 2), (5, 300)])
def test_gradient_field(E, ctx, shape):
    img = blurred_noise(shape, 3) if min(shape) > 2 else np.random.default_rng(4).random(shape).astype(np.float32)
    H, th = E.ecc_gradient_field(ctx, dev(img))
    check_field(host(H), host(th), img)


def test_gradient_field_batch_and_strides(E, ctx):
    import torch
    imgs = np.stack([blurred_noise((60, 70), 10 + b) for b in range(3)])
    H = torch.zeros((3, 60, 80), device="cuda")[:, :, :70]
    th = torch.zeros((3, 60, 80), device="cuda")[:, :, :70]
    E.ecc_gradient_field(ctx, dev(imgs), H, th)
    for b in range(3):
        check_field(host(H[b]), host(th[b]), imgs[b])


@pytest.mark.parametrize("which", ["matching_pattern", "random_31", "random_3"])
def test_voting_filter(E, ctx, which):
    if which == "matching_pattern":
        _, pat, _ = matching_scene(1024, 63)
    elif which == "random_31":
        pat = random_filter(31, 7, 6.0)
    else:
        pat = random_filter(3, 8, 1.0)
    F = host(E.ecc_voting_filter(ctx, dev(pat))).astype(np.float64)
    ref = O.voting_filter(pat)
    assert rel2(F, ref) <= 1e-6, rel2(F, ref)
    # every run gives the same bits
    assert np.array_equal(host(E.ecc_voting_filter(ctx, dev(pat))), F.astype(np.float32))


def peaks_equal(E, ctx, D, radius, thr, relative, max_peaks):
    rows, cols, vals = E.ecc_find_peaks(ctx, dev(D), radius, thr, relative, max_peaks)
    # the threshold as the library forms it: float32 arithmetic
    t = np.float32(thr) * np.float32(D.max()) if relative else np.float32(thr)
    rr, rc, rv = O.find_peaks(D.astype(np.float64), radius, float(t), max_peaks)
    assert host(rows).tolist() == rr.tolist()
    assert host(cols).tolist() == rc.tolist()
    assert np.array_equal(host(vals).astype(np.float64), rv)


@pytest.mark.parametrize("radius,thr,relative,max_peaks", [(3, 0.5, False, 1000), (8, 0.3, True, 10),
                                                           (0, 0.55, False, 50), (1, 0.95, True, 3),
                                                           (32, 0.2, True, 100), (40, 0.2, True, 100)])
def test_find_peaks_matches_the_oracle(E, ctx, radius, thr, relative, max_peaks):
    D = blurred_noise((150, 173), 21, sigma=1.5)
    peaks_equal(E, ctx, D, radius, thr, relative, max_peaks)


@pytest.mark.parametrize("shape,radius,thr,relative,max_peaks", [
    ((256, 256), 1, -10.0, False, 20000),   # every local maximum; 128^2 cells: the largest on-chip sort
    ((150, 173), 0, 0.5, True, 30000),      # 25950 cells: the device-wide sort, relative threshold
    ((300, 260), 2, 0.1, True, 5000)])
def test_find_peaks_long_lists(E, ctx, shape, radius, thr, relative, max_peaks):
    """Lists of thousands of peaks, in both sorts, with either threshold."""
    D = blurred_noise(shape, 23, sigma=1.0)
    peaks_equal(E, ctx, D, radius, thr, relative, max_peaks)


def test_find_peaks_ties_and_plateaus(E, ctx):
    D = np.zeros((40, 50), np.float32)
    D[10:13, 10:13] = 2.0          # a plateau: only its first pixel is a peak
    D[30, 5] = D[30, 8] = 1.5      # equal values within each other's window
    D[25, 40] = 1.5                # and one far away: ties by raster index
    peaks_equal(E, ctx, D, 4, 1.0, False, 10)


def test_detection_on_the_matching_scene(E, ctx):
    """The three strongest peaks of the GPU response are the three pasted centres, as the
    oracle finds them; the response agrees with the oracle's to 1e-5 (rel-L2)."""
    img, pat, truth = matching_scene(1024, 63)
    print("detection 1024^2, 63x63 pattern, K=16", flush=True)
    rows, cols, vals, D = E.detect_pattern(ctx, dev(img), dev(pat), 16, radius=8, threshold=0.3, max_peaks=3)
    got = sorted(zip(host(rows).tolist(), host(cols).tolist()))
    assert got == sorted((r, c) for r, c, _ in truth)
    ref, _ = O.detection_response(img, pat, 16)
    Dg = host(D).astype(np.float64)
    assert rel2(Dg, ref) <= 1e-5
    # peak lists of the GPU response, exact against the oracle's definition
    peaks_equal(E, ctx, host(D), 8, 0.2, True, 20)
