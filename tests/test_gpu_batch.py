"""Batch plans: each plane's result inside a ragged batch equals its result alone
(bit-exact: same kernels, integer reductions), and equals the oracle, in both
layouts (persistent strided workgroups, one workgroup per plane); captured
graphs give the same result on every replay."""
import re

import numpy as np
import pytest
import torch

import oracle as O
from paper_1402_6034_amd import synth

pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1402_6034_amd.rdct")
DEV = "cuda:0"
LAYOUTS = [R.LAYOUT_STRIDED, R.LAYOUT_PER_PLANE]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ragged_planes(n, seed, full_blocks=True):
    rng = np.random.default_rng(seed)
    shapes = []
    for i in range(n):
        h, w = int(rng.integers(1, 40)) * 8, int(rng.integers(1, 40)) * 8
        if not full_blocks and i % 3 == 0:
            h, w = h - int(rng.integers(0, 7)), w - int(rng.integers(0, 7))
        shapes.append((h, w))
    imgs = [synth.render_np(1000 * seed + i, h, w) for i, (h, w) in enumerate(shapes)]
    return imgs, [torch.from_numpy(a).to(DEV) for a in imgs], rng


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("full", [True, False])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_quant_batch_equals_single_and_oracle(full, use_graph, layout):
    imgs, dev, rng = ragged_planes(23, 1, full)
    quals = [int(q) for q in rng.integers(10, 91, size=len(imgs))]
    sels = [R.select(R.SEL_QUANT, quality=q, level_shift=128) for q in quals]
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True,
                       tuning=R.Tuning(1 + 3 * (layout == R.LAYOUT_PER_PLANE), 4, use_graph, layout))
    assert plan.tuning.layout == layout
    plan.run()
    sse = host(plan.sse)
    for i, (img, d, sel) in enumerate(zip(imgs, dev, sels)):
        s1, c1, r1 = R.compress_eval(d, sel, 1, R.COEF_I16, True)
        assert int(host(s1)[0]) == int(sse[i]), i
        assert np.array_equal(host(c1), host(plan.coef_views[i])), i
        assert np.array_equal(host(r1), host(plan.recon_views[i])), i
    for i in (0, 5, 11):
        ref = O.quant_eval(imgs[i], O.quant_table(quals[i]))
        assert np.array_equal(host(plan.coef_views[i]).astype(np.int64), ref["q"].reshape(-1, 64))
        assert np.max(np.abs(host(plan.recon_views[i]) - ref["recon"])) <= 1e-4
        h, w = imgs[i].shape
        assert abs(R.psnr_from_sse(int(sse[i]), R.SEL_QUANT, h, w) - ref["psnr"]) <= 1e-3
    plan.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_quant_batch_exact_ties(layout):
    # Small uniform tables make exact ties Y / (g_k Q) = n + 1/2 frequent where
    # s_k s_l is rational; they must round away from zero in both quantiser forms:
    # whole-block planes (coefficient-domain error) and planes with partial blocks
    # (pixel-domain error) in one batch.
    shapes = [(64, 64), (96, 80), (40, 128), (70, 50), (37, 61), (128, 72)]
    imgs = [synth.render_np(500 + i, h, w) for i, (h, w) in enumerate(shapes)]
    dev = [torch.from_numpy(a).to(DEV) for a in imgs]
    qvs = [1, 2, 3, 4, 5, 6]
    sels = [R.select(R.SEL_QUANT, qtable=[qv] * 64, level_shift=128) for qv in qvs]
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True,
                       tuning=R.Tuning(1 + 3 * (layout == R.LAYOUT_PER_PLANE), 4, 0, layout))
    plan.run()
    sse = host(plan.sse)
    g_ = np.diag(O.gram())
    rational = np.equal.outer(g_, g_)
    n_ties = 0
    for i, (img, qv) in enumerate(zip(imgs, qvs)):
        qt = np.full((8, 8), qv)
        ref = O.quant_eval(img, qt)
        y = np.asarray(ref["Y"])
        num = 2 * np.abs(y)
        den = np.where(rational, g_[:, None] * qv, 1) * np.ones((8, 8), dtype=np.int64)
        n_ties += int((rational & (num % den == 0) & ((num // den) % 2 == 1)).sum())
        assert np.array_equal(host(plan.coef_views[i]).astype(np.int64), ref["q"].reshape(-1, 64)), i
        assert np.max(np.abs(host(plan.recon_views[i]) - ref["recon"])) <= 1e-4, i
        h, w = img.shape
        assert abs(R.psnr_from_sse(int(sse[i]), R.SEL_QUANT, h, w) - ref["psnr"]) <= 1e-3, i
    assert n_ties > 100


@pytest.mark.parametrize("layout", LAYOUTS)
def test_retention_batch_equals_single_and_oracle(layout):
    imgs, dev, rng = ragged_planes(17, 2, full_blocks=False)
    rs = [int(r) for r in rng.integers(1, 46, size=len(imgs))]
    sels = [R.select(R.SEL_ZIGZAG, r=r) for r in rs]
    plan = R.BatchPlan(dev, sels, R.COEF_I32, recon=True, tuning=R.Tuning(2, 4, 1, layout))
    plan.run()
    sse = host(plan.sse)
    for i, (img, d, sel) in enumerate(zip(imgs, dev, sels)):
        s1, c1, r1 = R.compress_eval(d, sel, 1, R.COEF_I32, True)
        assert int(host(s1)[0]) == int(sse[i])
        assert np.array_equal(host(c1), host(plan.coef_views[i]))
        assert np.array_equal(host(r1), host(plan.recon_views[i]))
        ref = O.retention_eval(img, [rs[i]])
        assert int(sse[i]) == ref["sse_num"][rs[i]]
    plan.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_graph_replays_are_identical(layout):
    imgs, dev, rng = ragged_planes(9, 3)
    sels = [R.select(R.SEL_QUANT, quality=int(q), level_shift=128) for q in rng.integers(10, 91, 9)]
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True, tuning=R.Tuning(1, 2, 1, layout))
    plan.run()
    ref = (host(plan.sse).copy(), host(plan.coef).copy(), host(plan.recon).copy())
    for k in range(4):
        # Eager work between replays: scribble over the outputs.
        plan.coef.fill_(-7)
        plan.recon.fill_(float("nan"))
        plan.sse.fill_(123456789)
        torch.cuda.synchronize()
        plan.run()
        assert np.array_equal(host(plan.sse), ref[0]), k
        assert np.array_equal(host(plan.coef), ref[1]), k
        assert np.array_equal(host(plan.recon), ref[2]), k
    plan.close()


def test_autotune_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("RDCT_TUNING_CACHE", str(tmp_path / "tune.json"))
    imgs, dev, rng = ragged_planes(12, 4)
    sels = [R.select(R.SEL_QUANT, quality=50, level_shift=128) for _ in imgs]
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True)
    plan.run()
    before = host(plan.sse).copy()
    t = plan.autotune(reps=2)
    assert t.waves_per_wg in (1, 2, 4) and 1 <= t.wgs_per_cu <= 16 and t.layout in LAYOUTS
    plan.run()
    assert np.array_equal(host(plan.sse), before)
    text = (tmp_path / "tune.json").read_text()
    assert '"waves_per_wg"' in text and '"layout"' in text and "gfx950/batch" in text
    # A new plan of the same class picks the cached geometry.
    plan2 = R.BatchPlan(dev, sels, R.COEF_I16, recon=True)
    got = (plan2.tuning.waves_per_wg, plan2.tuning.wgs_per_cu, plan2.tuning.layout)
    assert got == (t.waves_per_wg, t.wgs_per_cu, t.layout)
    plan.close()
    plan2.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_batch_of_one_full_hd_plane_and_tiny_planes(layout):
    shapes = [(1080, 1920), (8, 8), (1, 1), (13, 7)]
    imgs = [synth.render_np(50 + i, h, w) for i, (h, w) in enumerate(shapes)]
    dev = [torch.from_numpy(a).to(DEV) for a in imgs]
    sels = [R.select(R.SEL_ZIGZAG, r=r) for r in (10, 1, 64, 3)]
    plan = R.BatchPlan(dev, sels, None, recon=False, tuning=R.Tuning(4, 2, 1, layout))
    plan.run()
    sse = host(plan.sse)
    for i, img in enumerate(imgs):
        r = sels[i].r
        s1, _, _ = R.compress_eval(dev[i], sels[i], 1)
        assert int(host(s1)[0]) == int(sse[i])
    ref = O.retention_eval(imgs[3], [3])
    assert int(sse[3]) == ref["sse_num"][3]
    plan.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("use_graph", [1, 0])
def test_sweep_batch_equals_single_and_oracle(use_graph, layout):
    imgs, dev, rng = ragged_planes(19, 5)
    count = 12
    r0s = [int(r) for r in rng.integers(1, 64 - count + 2, size=len(imgs))]
    r0s[3] = 64 - count + 1     # a range that ends at r = 64
    sels = [R.select(R.SEL_ZIGZAG, r=r) for r in r0s]
    plan = R.BatchPlan(dev, sels, R.COEF_I32, recon=True, r_count=count,
                       tuning=R.Tuning(2, 4, use_graph, layout))
    plan.sse.fill_(-1)          # every sum is written by a run
    for _ in range(2):          # twice: the sums are cleared by every run
        plan.run()
    sse = host(plan.sse)
    assert sse.shape == (len(imgs), count)
    for i, (img, d, sel) in enumerate(zip(imgs, dev, sels)):
        s1, c1, r1 = R.compress_eval(d, sel, count, R.COEF_I32, True)
        assert np.array_equal(host(s1), sse[i]), i
        assert np.array_equal(host(c1), host(plan.coef_views[i])), i
        assert np.array_equal(host(r1), host(plan.recon_views[i])), i
    assert sse[3][-1] == 0
    for i in (0, 3, 7, 18):
        rs = list(range(r0s[i], r0s[i] + count))
        ref = O.retention_eval(imgs[i], rs)
        assert [int(v) for v in sse[i]] == [ref["sse_num"][r] for r in rs], i
    plan.close()


def test_sweep_batch_rejects_partial_blocks():
    imgs, dev, _ = ragged_planes(3, 6)
    dev.append(torch.from_numpy(synth.render_np(7, 20, 24)).to(DEV))
    sels = [R.select(R.SEL_ZIGZAG, r=1) for _ in dev]
    with pytest.raises(R.RdctError):
        R.BatchPlan(dev, sels, None, r_count=45)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_many_tiny_planes(layout):
    """2000 planes of 1..24 pixels a side (one to nine blocks, partial blocks
    included): every plane's sum equals its own launch and, for a sample, the
    oracle; in the per-plane layout that is 2000 workgroups of one item each."""
    rng = np.random.default_rng(77)
    shapes = [(int(rng.integers(1, 25)), int(rng.integers(1, 25))) for _ in range(2000)]
    imgs = [synth.render_np(9000 + i, h, w) for i, (h, w) in enumerate(shapes)]
    dev = [torch.from_numpy(a).to(DEV) for a in imgs]
    quals = [int(q) for q in rng.integers(5, 96, size=len(imgs))]
    sels = [R.select(R.SEL_QUANT, quality=q, level_shift=128) for q in quals]
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True, tuning=R.Tuning(4, 4, 0, layout))
    plan.sse.fill_(-1)
    plan.run()
    sse = host(plan.sse)
    for i in rng.choice(len(imgs), size=60, replace=False):
        s1, c1, r1 = R.compress_eval(dev[i], sels[i], 1, R.COEF_I16, True)
        assert int(host(s1)[0]) == int(sse[i]), i
        assert np.array_equal(host(c1), host(plan.coef_views[i])), i
        assert np.array_equal(host(r1), host(plan.recon_views[i])), i
    for i in range(0, len(imgs), 97):
        ref = O.quant_eval(imgs[i], O.quant_table(quals[i]), level_shift=128)
        assert np.array_equal(host(plan.coef_views[i]).astype(np.int64), ref["q"].reshape(-1, 64)), i
        assert np.max(np.abs(host(plan.recon_views[i]) - ref["recon"])) <= 1e-4, i
    plan.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_many_small_sweep_planes(layout):
    """1500 whole-block planes of 8..32 pixels a side, retention sweep over the
    full r = 20..64 range in one launch, against the oracle for a sample."""
    rng = np.random.default_rng(78)
    shapes = [(8 * int(rng.integers(1, 5)), 8 * int(rng.integers(1, 5))) for _ in range(1500)]
    imgs = [synth.render_np(12000 + i, h, w) for i, (h, w) in enumerate(shapes)]
    dev = [torch.from_numpy(a).to(DEV) for a in imgs]
    count = 45
    sels = [R.select(R.SEL_ZIGZAG, r=20)] * len(imgs)
    plan = R.BatchPlan(dev, sels, None, recon=False, r_count=count,
                       tuning=R.Tuning(2, 8, 0, layout))
    plan.sse.fill_(-1)
    plan.run()
    sse = host(plan.sse)
    assert np.all(sse[:, -1] == 0)                      # r = 64 keeps everything
    for i in range(0, len(imgs), 53):
        ref = O.retention_eval(imgs[i], range(20, 65))
        assert [int(v) for v in sse[i]] == [ref["sse_num"][r] for r in range(20, 65)], i
    plan.close()


@pytest.mark.parametrize("xcd,strip", [(0, 1), (1, 1), (1, 2), (0, 4), (1, 8)])
@pytest.mark.parametrize("wpg,wpc", [(1, 4), (2, 3), (4, 1)])
def test_xcd_ranges_and_strips_give_identical_outputs(xcd, strip, wpg, wpc):
    # The XCD-range order and the strip of the strided layout change which wave
    # runs which item, never a result: every output equals the single-plane
    # call's.
    imgs, dev, rng = ragged_planes(37, 9, full_blocks=False)
    quals = [int(q) for q in rng.integers(10, 91, size=len(imgs))]
    sels = [R.select(R.SEL_QUANT, quality=q, level_shift=128) for q in quals]
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True,
                       tuning=R.Tuning(wpg, wpc, 0, R.LAYOUT_STRIDED, xcd, strip))
    assert plan.tuning.xcd_ranges == xcd and plan.tuning.strip == strip
    for _ in range(2):
        plan.run()
    sse = host(plan.sse)
    for i, (d, sel) in enumerate(zip(dev, sels)):
        s1, c1, r1 = R.compress_eval(d, sel, 1, R.COEF_I16, True)
        assert int(host(s1)[0]) == int(sse[i]), i
        assert np.array_equal(host(c1), host(plan.coef_views[i])), i
        assert np.array_equal(host(r1), host(plan.recon_views[i])), i
    # A geometry set on the existing plan (here graph replay, the other XCD
    # order and the per-plane layout) gives the same outputs.
    coef0, recon0 = host(plan.coef).copy(), host(plan.recon).copy()
    for t in (R.Tuning(wpg, wpc, 1, R.LAYOUT_STRIDED, 1 - xcd, 1 if strip > 1 else 4),
              R.Tuning(4, 1, 0, R.LAYOUT_PER_PLANE, 0)):
        plan.set_tuning(t)
        plan.sse.fill_(7)
        plan.run()
        plan.run()
        assert np.array_equal(host(plan.sse), sse)
        assert np.array_equal(host(plan.coef), coef0) and np.array_equal(host(plan.recon), recon0)
    for bad in (R.Tuning(3, 4, 0, R.LAYOUT_STRIDED, 0), R.Tuning(1, 4, 0, R.LAYOUT_STRIDED, 1, 3)):
        with pytest.raises(R.RdctError):
            plan.set_tuning(bad)
    plan.close()


@pytest.mark.parametrize("tuning", [(3, 4, 0, 1), (1, 17, 0, 1), (1, 4, 0, 3), (2, 0, 0, -1),
                                    (1, 4, 0, 1, 2), (1, 4, 0, 1, 1, 16), (1, 4, 0, 1, 1, -2)])
def test_invalid_tuning_rejected(tuning):
    """Waves per workgroup outside 1, 2, 4, resident workgroups outside 1..16,
    unknown layouts, XCD-range flags other than 0 and 1 and strips other than
    1, 2, 4, 8 are refused at plan creation (nothing is launched)."""
    imgs, dev, _ = ragged_planes(2, 8)
    sels = [R.select(R.SEL_ZIGZAG, r=5)] * 2
    with pytest.raises(R.RdctError) as e:
        R.BatchPlan(dev, sels, None, tuning=R.Tuning(*tuning))
    assert e.value.status == R.ERR_INVALID_ARG


def test_invalid_cache_entry_is_ignored(tmp_path, monkeypatch):
    """A tuning-cache entry that is not a valid geometry (edited by hand, or from
    another build) is skipped: the plan takes the default geometry."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("RDCT_TUNING_CACHE", str(cache))
    imgs, dev, _ = ragged_planes(6, 9)
    sels = [R.select(R.SEL_QUANT, quality=50, level_shift=128)] * len(dev)
    plan = R.BatchPlan(dev, sels, R.COEF_I16, recon=True)
    plan.autotune(reps=1)
    plan.run()
    want = host(plan.sse).copy()
    plan.close()
    text = cache.read_text()
    cache.write_text(re.sub(r'"waves_per_wg": \d+', '"waves_per_wg": 3', text))
    plan2 = R.BatchPlan(dev, sels, R.COEF_I16, recon=True)
    t = plan2.tuning
    assert (t.waves_per_wg, t.wgs_per_cu, t.layout, t.use_graph) == (1, 8, R.LAYOUT_STRIDED, 0)
    plan2.run()
    assert np.array_equal(host(plan2.sse), want)
    plan2.close()
