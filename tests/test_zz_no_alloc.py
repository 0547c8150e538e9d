"""The matching entry point that allocates nothing, against ecc_match_rotations.

Both run the same kernels on the same values (the no-allocation form only splits the
component stack into bands of block rows that pass through a fixed device array), so
scores and indices must agree exactly. Two calls in a row, the second on a smaller,
ragged image; a call before the plan has its block spectra is refused on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import paper_2006_13188_amd as E
    return E


def _run_pair(E, ctx, plan, img, prec):
    import torch
    H = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    ref_s, ref_i = E.ecc_match_rotations(ctx, plan, H, 64, prec)
    s = torch.full(H.shape, -7.0, dtype=torch.float32, device="cuda")
    i = torch.full(H.shape, -7, dtype=torch.int32, device="cuda")
    E.ecc_match_rotations_noalloc(ctx, plan, H, s, i, 64, prec)
    torch.cuda.synchronize()
    return ref_s.cpu().numpy(), ref_i.cpu().numpy(), s.cpu().numpy(), i.cpu().numpy()


@pytest.mark.parametrize("prec_name", ["PREC_FP32", "PREC_MFMA_FP16_HILO"])
def test_noalloc_matches_allocating_call(E, prec_name):
    import torch
    from synthetic import matching_scene
    prec = getattr(E, prec_name)
    img, pat, _ = matching_scene(1024, 63)
    ctx = E.Context(0)
    plan = E.FilterPlan.rotation(ctx, torch.from_numpy(pat).cuda(), 16)
    try:
        # 1024^2, 17 components, 64-row blocks: 8.9 MB per block row, several bands
        print(f"noalloc {prec_name}: 1024x1024 scene, 63x63 pattern, K=16", flush=True)
        rs, ri, s, i = _run_pair(E, ctx, plan, img, prec)
        assert np.array_equal(rs, s) and np.array_equal(ri, i)
        # second call, smaller and ragged (a partial last block row and column)
        print(f"noalloc {prec_name}: 300x517 crop", flush=True)
        rs, ri, s, i = _run_pair(E, ctx, plan, img[100:400, 200:717], prec)
        assert np.array_equal(rs, s) and np.array_equal(ri, i)
    finally:
        plan.close()
        ctx.close()


def test_noalloc_refuses_a_plan_without_block_spectra(E):
    import torch
    from synthetic import random_filter
    ctx = E.Context(0)
    plan = E.FilterPlan.rotation(ctx, torch.from_numpy(random_filter(31, 5, 8.0)).cuda(), 8)
    try:
        H = torch.zeros((256, 256), dtype=torch.float32, device="cuda")
        s = torch.zeros_like(H)
        i = torch.zeros((256, 256), dtype=torch.int32, device="cuda")
        with pytest.raises(E.EccError) as ei:
            E.ecc_match_rotations_noalloc(ctx, plan, H, s, i, 64)
        assert ei.value.status == 2
    finally:
        plan.close()
        ctx.close()
