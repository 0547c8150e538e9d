"""Steering in 3D (Sec. 9) on the GPU against the float64 oracle.

* plan components (device spherical-harmonic transform per radius) against the oracle's;
* whole correlation / convolution against closed forms (a filter linear in the
  coordinates under a random rotation field);
* random filters and fields against the oracle's FFT route on volumes that span several
  transform radices with ragged sizes, K = 0..4, degenerate thin volumes;
* the 128^3 volume, 15^3 filter, K = 4 configuration at sampled voxels (corners and
  edges included), each checked against the oracle run on the crop of the volume that
  the voxel's value depends on.
Tolerance: rel-L2 and rel-inf <= 1e-5 (float32 transforms, float64 spectra and
Wigner-D)."""
import numpy as np
import pytest

from oracle import steer3d as O3
from synthetic import steer3d_config

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
    return t.detach().cpu().numpy()


def run(E, ctx, op, plan, vol, a, b, g):
    return host(E.ecc_extended_3d(ctx, op, plan, dev(vol), dev(a), dev(b), dev(g))).astype(np.float64)


@pytest.mark.parametrize("S,K", [(5, 2), (7, 3), (9, 4), (15, 4), (7, 0)])
def test_plan_components_match_the_oracle(E, ctx, S, K):
    _, filt, *_ = steer3d_config((4, 4, 4), S, seeds=(1, 2 + S, 3))
    plan = E.VolumePlan(ctx, dev(filt), K)
    comps, table, w = plan.components()
    hs, ref = O3.components3d(filt.astype(np.float64), K)
    assert plan.U == len(hs)
    assert table.tolist() == [[l, mp, m] for l, mp, m, _ in hs]
    assert w.tolist() == [h[3] for h in hs]
    got = host(comps).astype(np.complex128)
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))
    plan.close()


def closed_form(vol, a, b, g, S, op):
    coef = np.array([0.3, -1.1, 0.7])
    Rm = O3.euler_matrix(a, b, g)
    R = (S - 1) // 2
    d = np.arange(-R, R + 1, dtype=np.float64)
    z, y, x = np.meshgrid(d, d, d, indexing="ij")
    q = np.stack([x, y, z], -1)
    ball = (x * x + y * y + z * z) <= R * R
    nz, ny, nx = vol.shape
    V = vol.astype(np.float64)
    if op == 0:
        Hp = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
        Hp[R:R + nz, R:R + ny, R:R + nx] = V
        out = np.zeros(V.shape)
        for k in range(nz):
            for i in range(ny):
                for j in range(nx):
                    f = np.where(ball, (q @ Rm[k, i, j]) @ coef, 0.0)
                    out[k, i, j] = np.sum(Hp[k:k + S, i:i + S, j:j + S] * f)
        return out
    yp = np.zeros((nz + 2 * R, ny + 2 * R, nx + 2 * R))
    for k in range(nz):
        for i in range(ny):
            for j in range(nx):
                yp[k:k + S, i:i + S, j:j + S] += V[k, i, j] * np.where(ball, (q @ Rm[k, i, j]) @ coef, 0.0)
    return yp[R:R + nz, R:R + ny, R:R + nx]


@pytest.mark.parametrize("op", [0, 1])
def test_linear_filter_closed_form(E, ctx, op):
    S = 7
    vol, _, a, b, g = steer3d_config((9, 10, 11), S, seeds=(5, 6, 7))
    R = (S - 1) // 2
    d = np.arange(-R, R + 1, dtype=np.float64)
    z, y, x = np.meshgrid(d, d, d, indexing="ij")
    filt = (0.3 * x - 1.1 * y + 0.7 * z).astype(np.float32)
    ref = closed_form(vol, a.astype(np.float64), b.astype(np.float64), g.astype(np.float64), S, op)
    for K in (1, 3):
        plan = E.VolumePlan(ctx, dev(filt), K)
        got = run(E, ctx, op, plan, vol, a, b, g)
        assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (K, rel2(got, ref), relinf(got, ref))
        plan.close()


CASES = [((20, 22, 24), 7, 3), ((17, 13, 29), 9, 4), ((24, 24, 24), 5, 2), ((1, 6, 9), 5, 2), ((11, 1, 1), 3, 1),
         ((12, 14, 10), 7, 0), ((2, 3, 4), 15, 2), ((9, 11, 10), 9, 6), ((8, 7, 9), 7, 8), ((16, 12, 14), 11, 5),
         # transform lengths of 135 (compiled schedule) along z, then along y and x
         ((128, 6, 7), 15, 4), ((5, 128, 128), 15, 3)]


@pytest.mark.parametrize("shape,S,K", CASES)
@pytest.mark.parametrize("op", [0, 1])
def test_random_filter_matches_the_oracle(E, ctx, shape, S, K, op):
    vol, filt, a, b, g = steer3d_config(shape, S, seeds=(10 + S, 20 + K, 30))
    f64 = [v.astype(np.float64) for v in (vol, a, b, g)]
    ref = (O3.ext_corr3d_fft if op == 0 else O3.ext_conv3d_fft)(f64[0], f64[1], f64[2], f64[3],
                                                               filt.astype(np.float64), K)
    plan = E.VolumePlan(ctx, dev(filt), K)
    got = run(E, ctx, op, plan, vol, a, b, g)
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    # the same bits on a second call, and the workspace the call took is what the size query says
    again = run(E, ctx, op, plan, vol, a, b, g)
    assert np.array_equal(got, again)
    assert ctx.workspace_allocated() >= ctx.volume_workspace_size(plan, *shape)
    plan.close()


def crop_value(vol, a, b, g, filt, K, p, op, parts):
    """The oracle's value at voxel p from the crop that holds every voxel within R of p
    (zero outside the volume, as the operator's boundary)."""
    S = filt.shape[0]
    R = (S - 1) // 2
    lo = [max(0, c - R) for c in p]
    hi = [min(n, c + R + 1) for c, n in zip(p, vol.shape)]
    sl = tuple(slice(x0, x1) for x0, x1 in zip(lo, hi))
    f = O3.ext_corr3d_fft if op == 0 else O3.ext_conv3d_fft
    y = f(vol[sl].astype(np.float64), a[sl].astype(np.float64), b[sl].astype(np.float64),
          g[sl].astype(np.float64), filt.astype(np.float64), K, parts=parts)
    return y[tuple(c - x0 for c, x0 in zip(p, lo))]


@pytest.mark.parametrize("op", [0, 1])
def test_full_size_sampled(E, ctx, op):
    n, S, K = 128, 15, 4
    print(f"steer3d full size {n}^3, S={S}, K={K}, op={op}", flush=True)
    vol, filt, a, b, g = steer3d_config(n, S)
    plan = E.VolumePlan(ctx, dev(filt), K)
    got = run(E, ctx, op, plan, vol, a, b, g)
    rng = np.random.default_rng(77 + op)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5), (n // 2, 0, n - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(8)]
    parts = O3.components3d(filt.astype(np.float64), K)
    ref = np.array([crop_value(vol, a, b, g, filt, K, p, op, parts) for p in pts])
    val = np.array([got[p] for p in pts])
    scale_ = np.max(np.abs(got))
    assert np.max(np.abs(val - ref)) <= TOL * scale_, (np.max(np.abs(val - ref)) / scale_)
    assert np.all(np.isfinite(got))
    plan.close()


def test_invalid_arguments(E, ctx):
    import torch
    filt = dev(np.ones((7, 7, 7)))
    with pytest.raises(E.EccError):
        E.VolumePlan(ctx, filt, 9)                      # K beyond 8
    with pytest.raises(E.EccError):
        E.VolumePlan(ctx, dev(np.ones((6, 6, 6))), 2)   # even side
    plan = E.VolumePlan(ctx, filt, 2)
    v = torch.zeros((4, 5, 6), device="cuda")
    with pytest.raises(E.EccError):
        E.ecc_extended_3d(ctx, 0, plan, v, v, v, v, out=v)          # out aliases the inputs
    with pytest.raises(E.EccError):
        E.ecc_extended_3d(ctx, 0, plan, *(torch.zeros((0, 5, 6), device="cuda"),) * 4)   # empty volume
    plan.close()
