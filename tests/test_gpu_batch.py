"""Batched execution (many uneven correlations and convolutions in one captured graph)
against the float64 oracle and against one call per instance.

Instances have different image shapes (square and rectangular, ragged against every
block size), filter sizes 7..63 and band limits; three convolutions of different block
shapes go into the graph too, and one filter too large for a block shape exercises the
per-call remainder. The graph is replayed several times with unrelated eager GPU work in
between, and every replay is checked. Tolerance: rel-L2 and rel-inf <= 1e-5 against the
oracle."""
import numpy as np
import pytest

import oracle as O
from synthetic import batch_instance

pytestmark = pytest.mark.gpu
TOL = 1e-5

SHAPES = [(64, 64, 7, 4), (97, 130, 15, 6), (200, 173, 21, 10), (130, 90, 63, 12), (75, 75, 9, 3),
          (160, 230, 31, 16), (66, 201, 35, 8), (128, 128, 13, 24), (99, 64, 41, 5), (181, 77, 11, 7)]
CONV_SHAPES = [(90, 100, 15, 5), (150, 131, 9, 3), (140, 170, 41, 6)]


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
def setup(E):
    import torch
    ctx = E.Context(0)
    data, insts, refs = [], [], []
    for i, (ny, nx, S, K) in enumerate(SHAPES):
        img, filt, th = batch_instance(i, ny, nx, S)
        plan = E.FilterPlan.rotation(ctx, torch.from_numpy(filt).cuda(), K)
        H, T = torch.from_numpy(img).cuda(), torch.from_numpy(th).cuda()
        out = torch.full((ny, nx), float("nan"), device="cuda")
        comps, _ = O.angular_components(filt, K)
        refs.append(O.ext_corr_half(img.astype(np.float64), th.astype(np.float64), O.half_components(comps)))
        insts.append((E.CORRELATION, plan, H, T, out))
        data.append((img, filt, th, K))
    # convolutions (in the graph; block shapes 64, 96 and 128)
    for i, (ny, nx, S, K) in enumerate(CONV_SHAPES):
        img, filt, th = batch_instance(51 + i, ny, nx, S)
        plan = E.FilterPlan.rotation(ctx, torch.from_numpy(filt).cuda(), K)
        comps, _ = O.angular_components(filt, K)
        out = torch.full((ny, nx), float("nan"), device="cuda")
        insts.append((E.CONVOLUTION, plan, torch.from_numpy(img).cuda(), torch.from_numpy(th).cuda(), out))
        refs.append(O.ext_conv_half(img.astype(np.float64), th.astype(np.float64), O.half_components(comps)))
    # per-call remainder: a filter with no block shape (R = 60)
    img, filt, th = batch_instance(50, 130, 140, 121)
    plan = E.FilterPlan.rotation(ctx, torch.from_numpy(filt).cuda(), 3)
    comps, _ = O.angular_components(filt, 3)
    out = torch.full((130, 140), float("nan"), device="cuda")
    insts.append((E.CORRELATION, plan, torch.from_numpy(img).cuda(), torch.from_numpy(th).cuda(), out))
    refs.append(O.ext_corr_half(img.astype(np.float64), th.astype(np.float64), O.half_components(comps)))
    yield ctx, insts, refs
    ctx.close()


def check_all(insts, refs):
    import torch
    torch.cuda.synchronize()
    for (op, plan, H, T, out), ref in zip(insts, refs):
        y = out.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(y))
        assert rel2(y, ref) <= TOL and relinf(y, ref) <= TOL, (H.shape, rel2(y, ref), relinf(y, ref))


@pytest.mark.parametrize("flags", [0, 1, 2, 3], ids=["table", "table_autotune", "persistent",
                                                     "persistent_autotune"])
def test_batch_matches_oracle_over_replays(E, setup, flags):
    import torch
    ctx, insts, refs = setup
    for *_, out in insts:
        out.fill_(float("nan"))
    bp = E.BatchPlan(ctx, insts, flags)
    info = bp.info()
    assert info["graph_instances"] == len(SHAPES) + len(CONV_SHAPES) and 2 <= info["launches"] <= 9
    for rep in range(3):
        for *_, out in insts:
            out.fill_(float("nan"))
        bp.execute()
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")   # eager work
        check_all(insts, refs)
        assert torch.isfinite(junk).all()
    bp.close()


def test_persistent_batch_runs_several_items_per_workgroup(E):
    """More blocks than resident workgroups (8 x 121 blocks of 64 x 64), so the persistent
    workgroups loop over the item counter; replayed three times (the counter pair resets
    itself at the end of every launch) and checked against the oracle each time."""
    import torch
    ctx = E.Context(0)
    insts, refs = [], []
    for i in range(8):
        img, filt, th = batch_instance(100 + i, 700, 700, 31)
        plan = E.FilterPlan.rotation(ctx, torch.from_numpy(filt).cuda(), 6)
        comps, _ = O.angular_components(filt, 6)
        refs.append(O.ext_corr_half(img.astype(np.float64), th.astype(np.float64), O.half_components(comps)))
        out = torch.full((700, 700), float("nan"), device="cuda")
        insts.append((E.CORRELATION, plan, torch.from_numpy(img).cuda(), torch.from_numpy(th).cuda(), out))
    bp = E.BatchPlan(ctx, insts, E.BATCH_PERSISTENT)
    assert bp.info()["blocks"] > 2 * 256
    for rep in range(3):
        for *_, out in insts:
            out.fill_(float("nan"))
        bp.execute()
        check_all(insts, refs)
    bp.close()
    ctx.close()


def test_batch_agrees_with_per_call(E, setup):
    """One call per instance gives the same values (the block shape chosen for a lone
    call may differ from the batch's, so up to float32 rounding)."""
    import torch
    ctx, insts, refs = setup
    bp = E.BatchPlan(ctx, insts, 0)
    bp.execute()
    torch.cuda.synchronize()
    for op, plan, H, T, out in insts:
        y = E.ecc_extended(ctx, op, plan, H, T)
        torch.cuda.synchronize()
        assert float((y - out).abs().max()) <= 1e-6 * float(out.abs().max())
    bp.close()


def test_batch_update_pointers(E, setup):
    import torch
    ctx, insts, refs = setup
    bp = E.BatchPlan(ctx, insts, 0)
    outs2 = [torch.full_like(o, float("nan")) for *_, o in insts]
    insts2 = [(op, plan, H, T, o2) for (op, plan, H, T, _), o2 in zip(insts, outs2)]
    bp.update(insts2)
    bp.execute()
    check_all(insts2, refs)
    with pytest.raises(E.EccError):
        bp.update(insts2[:-1])                       # count differs
    bad = list(insts2)
    op, plan, H, T, o = bad[0]
    bad[0] = (op, plan, H[:-1], T[:-1], o[:-1])      # size differs
    with pytest.raises(E.EccError):
        bp.update(bad)
    bp.close()


def test_empty_and_invalid_batches(E, setup):
    import torch
    ctx, insts, refs = setup
    bp = E.BatchPlan(ctx, [], 0)
    bp.execute()
    assert bp.info() == {"graph_instances": 0, "launches": 0, "blocks": 0}
    bp.close()
    op, plan, H, T, out = insts[0]
    with pytest.raises(E.EccError):
        E.BatchPlan(ctx, [(op, plan, H, T, H)], 0)   # aliasing
    with pytest.raises(E.EccError):
        E.BatchPlan(ctx, [(op, plan, H, T, out)], 64)   # unknown flag


@pytest.mark.parametrize("direct", [False, True], ids=["auto", "direct"])
def test_batch_with_direct_instances(E, direct):
    """Small filters take the direct sums inside the graph, correlations and convolutions:
    S = 3 and 5 under AUTO (the time model prefers them there), every side up to 15 under
    DIRECT; the larger filter keeps its block shape in both (a single call of it under
    DIRECT is refused). Replayed twice, each replay against the oracle."""
    import torch
    ctx = E.Context(0)
    if direct:
        ctx.set_strategy(E.STRATEGY_DIRECT)
    specs = [(0, 70, 90, 3, 2), (0, 130, 64, 5, 6), (0, 48, 200, 11, 4), (0, 100, 100, 21, 5),
             (1, 60, 80, 5, 3), (1, 75, 66, 11, 2)]
    insts, refs = [], []
    for i, (op, ny, nx, S, K) in enumerate(specs):
        img, filt, th = batch_instance(200 + i, ny, nx, S)
        plan = E.FilterPlan.rotation(ctx, torch.from_numpy(filt).cuda(), K)
        comps, _ = O.angular_components(filt, K)
        f = O.ext_corr_half if op == 0 else O.ext_conv_half
        refs.append(f(img.astype(np.float64), th.astype(np.float64), O.half_components(comps)))
        out = torch.full((ny, nx), float("nan"), device="cuda")
        insts.append((op, plan, torch.from_numpy(img).cuda(), torch.from_numpy(th).cuda(), out))
        if direct and S > 15:
            with pytest.raises(E.EccError):
                ctx.describe(op, plan, ny, nx)
        else:
            want = E.STRATEGY_DIRECT if (S <= 5 or direct) else E.STRATEGY_TILED
            assert ctx.describe(op, plan, ny, nx)[0] == want
    bp = E.BatchPlan(ctx, insts, 0)
    info = bp.info()
    assert info["graph_instances"] == len(specs) and info["launches"] >= 3
    for rep in range(2):
        for *_, out in insts:
            out.fill_(float("nan"))
        bp.execute()
        check_all(insts, refs)
    bp.close()
    ctx.close()


def test_autotune_measurements_move_between_contexts(E):
    """The autotuner's block-shape costs exported as JSON from one context and imported
    into another give the same choices without measuring again; text from another kind of
    device, or missing a shape, is refused and leaves the context as it was."""
    import json
    import torch
    a = E.Context(0)
    with pytest.raises(E.EccError):
        a.autotune_export()                      # nothing measured yet
    a.set_autotune(True)
    _, filt, _ = batch_instance(300, 64, 64, 31)
    plan_a = E.FilterPlan.rotation(a, torch.from_numpy(filt).cuda(), 16)
    a.describe(E.CORRELATION, plan_a, 1024, 1024)   # measures
    text = a.autotune_export()
    d = json.loads(text)
    assert d["device"].startswith("gfx") and len(d["tile_cost"]) >= 3
    b = E.Context(0)
    b.set_autotune(True)
    bad = dict(d, device="gfx000")
    with pytest.raises(E.EccError):
        b.autotune_import(json.dumps(bad))
    with pytest.raises(E.EccError):
        b.autotune_import(json.dumps(dict(d, tile_cost=d["tile_cost"][:-1])))
    with pytest.raises(E.EccError):
        b.autotune_export()                      # still unmeasured after the refusals
    b.autotune_import(text)
    assert b.autotune_export() == text
    plan_b = E.FilterPlan.rotation(b, torch.from_numpy(filt).cuda(), 16)
    for ny, nx, K in ((1024, 1024, 16), (300, 500, 4), (2048, 700, 24)):
        assert a.describe(E.CORRELATION, plan_a, ny, nx) == b.describe(E.CORRELATION, plan_b, ny, nx)
    plan_a.close()
    plan_b.close()
    a.close()
    b.close()


def test_autotuned_fft_size(E):
    """With the autotuner on, the two-pass FFT size of (n, R) is one of the 7-smooth sizes
    from the smallest admissible one up to 1/8 above it, chosen once (cached); a two-pass
    correlation at the chosen sizes matches the oracle; the choices travel in the JSON."""
    import json
    import torch

    def smooth7(m):
        for f in (2, 3, 5, 7):
            while m % f == 0:
                m //= f
        return m == 1

    plain = E.Context(0)
    c = E.Context(0)
    c.set_autotune(True)
    c.set_strategy(E.STRATEGY_TWO_PASS)
    for n, R in ((1000, 15), (700, 15), (1500, 31), (100, 3)):
        Pmin = plain.fft_size(n, R)
        P = c.fft_size(n, R)
        assert smooth7(P) and Pmin <= P and 8 * P <= 9 * Pmin, (n, R, Pmin, P)
        assert c.fft_size(n, R) == P
    ny, nx, S, K = 700, 1000, 31, 6
    img, filt, th = batch_instance(400, ny, nx, S)
    plan = E.FilterPlan.rotation(c, torch.from_numpy(filt).cuda(), K)
    y = E.ecc_extended(c, E.CORRELATION, plan, torch.from_numpy(img).cuda(), torch.from_numpy(th).cuda())
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    comps, _ = O.angular_components(filt, K)
    ref = O.ext_corr_half(img.astype(np.float64), th.astype(np.float64), O.half_components(comps))
    assert rel2(got, ref) <= TOL and relinf(got, ref) <= TOL, (rel2(got, ref), relinf(got, ref))
    text = c.autotune_export()
    sizes = {(a, b): p for a, b, p in json.loads(text)["fft_size"]}
    assert sizes[(1000, 15)] == c.fft_size(1000, 15) and sizes[(700, 15)] == c.fft_size(700, 15)
    d = E.Context(0)
    d.set_autotune(True)
    d.autotune_import(text)
    for (a, b), p in sizes.items():
        assert d.fft_size(a, b) == p
    plan.close()
    for x in (plain, c, d):
        x.close()
