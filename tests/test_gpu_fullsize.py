"""Parity at the benchmark workloads' full sizes, in the launch configurations
bench.py times: sampled blocks against the oracle, block by block, and
size-independent properties (batch == single plane, sums over blocks).

  * frame   8192 x 8192, quality 50, int16 q (single-plane kernel), and its
            inverse back to float32 pixels
  * ragged  the 1000-plane batch (persistent kernel, default geometry and the
            autotuned one), int16 q + float32 reconstruction + per-plane SSE
  * sweep   256 planes of 512 x 512, keep r = 1..45 (one batch launch, and
            one launch per plane)
  * codec   the 8192 x 8192 frame through encode + pack
  * comparison  one plan per transform over the sweep's 256 planes, r = 1..45
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1402_6034_amd import synth

pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1402_6034_amd.rdct")
DEV = "cuda:0"


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sample_idx(rng, nb, k):
    idx = np.unique(np.concatenate([[0, nb - 1], rng.integers(0, nb, size=k)]))
    return idx


@pytest.fixture(scope="module")
def frame():
    img = synth.render(0, 8192, 8192, device=DEV)
    return img, host(img)


def oracle_q_blocks(img_np, idx, quality, shift=128):
    blocks = O.sample_blocks(img_np, idx)
    y = O.forward_blocks(blocks, shift)
    return O.quantize(y, O.quant_table(quality)), y


def test_frame_quantise_sampled(frame):
    img, img_np = frame
    sel = R.select(R.SEL_QUANT, quality=50, level_shift=128)
    q = R.forward(img, sel, R.COEF_I16)
    nb = 1024 * 1024
    idx = sample_idx(np.random.default_rng(0), nb, 3000)
    want, _ = oracle_q_blocks(img_np, idx, 50)
    got = host(q[torch.from_numpy(idx).to(DEV)]).astype(np.int64)
    assert np.array_equal(got, want.reshape(-1, 64))


def test_inverse_frame_sampled(frame):
    # rdct_inverse as the inverse workload times it: the frame's Q50 int16 q back
    # to float32 pixels (staged row stores), sampled blocks against the oracle's
    # float64 dequantise + C_orth^T Z C_orth + 128, within 1e-4.
    img, img_np = frame
    sel = R.select(R.SEL_QUANT, quality=50, level_shift=128)
    q = R.forward(img, sel, R.COEF_I16)
    rec = R.inverse(q, 8192, 8192, sel, R.COEF_I16)
    nb = 1024 * 1024
    idx = sample_idx(np.random.default_rng(4), nb, 3000)
    want_q, _ = oracle_q_blocks(img_np, idx, 50)
    want = O.inverse_orth(O.dequantize(want_q, O.quant_table(50))) + 128
    by, bx = idx // 1024, idx % 1024
    r = host(rec)
    got = np.stack([r[8 * y:8 * y + 8, 8 * x:8 * x + 8] for y, x in zip(by, bx)])
    assert float(np.max(np.abs(got - want))) <= 1e-4


def test_codec_frame_sampled(frame):
    img, img_np = frame
    c = R.Codec(8192, 8192, DEV)
    c.encode(img, R.select(R.SEL_QUANT, quality=50, level_shift=128))
    c.pack()
    torch.cuda.synchronize()
    nb = 1024 * 1024
    counts = host(c.counts).astype(np.int64) & 0xffff
    off = host(c.offsets).astype(np.int64)
    assert off[0] == 0 and np.array_equal(np.diff(off), counts)
    idx = sample_idx(np.random.default_rng(1), nb, 1500)
    q, _ = oracle_q_blocks(img_np, idx, 50)
    words = host(c.packed).astype(np.int64) & 0xffffffff
    recon = host(c.recon)
    qt = O.quant_table(50)
    for n, b in enumerate(idx):
        pairs = O.rle_encode(O.zigzag_scan(q[n], 64))
        w = words[off[b]:off[b + 1]]
        assert list(zip((w >> 16).tolist(), (((w & 0xffff) ^ 0x8000) - 0x8000).tolist())) == pairs
        rec = O.inverse_orth(O.dequantize(q[n], qt)) + 128
        by, bx = divmod(int(b), 1024)
        got = recon[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8]
        near = np.abs(np.abs(rec - np.floor(rec)) - 0.5) < 1e-9
        assert np.array_equal(got[~near], O.u8_from_float(rec)[~near])


@pytest.fixture(scope="module")
def ragged():
    items = synth.ragged_batch(0, 1000)
    imgs = [synth.render(it.seed, it.height, it.width, device=DEV) for it in items]
    sels = [R.select(R.SEL_QUANT, quality=it.quality, level_shift=128) for it in items]
    return items, imgs, sels


@pytest.mark.parametrize("mode", ["default", "autotune", "per-plane"])
def test_ragged_batch_sampled(ragged, mode, tmp_path, monkeypatch):
    monkeypatch.setenv("RDCT_TUNING_CACHE", str(tmp_path / "tune.json"))
    items, imgs, sels = ragged
    tuning = R.Tuning(4, 1, 0, R.LAYOUT_PER_PLANE) if mode == "per-plane" else None
    plan = R.BatchPlan(imgs, sels, R.COEF_I16, recon=True, tuning=tuning)
    if mode == "autotune":
        plan.autotune(reps=2)
    plan.run()
    sse = host(plan.sse)
    rng = np.random.default_rng(2)
    order = np.argsort([it.height * it.width for it in items])
    for i in list(order[:40]) + list(rng.choice(1000, size=40, replace=False)):
        it, img_np = items[i], host(imgs[i])
        h, w = img_np.shape
        nb = (h // 8) * (w // 8)
        idx = sample_idx(rng, nb, 16)
        want_q, _ = oracle_q_blocks(img_np, idx, it.quality)
        got_q = host(plan.coef_views[i][torch.from_numpy(idx).to(DEV)]).astype(np.int64)
        assert np.array_equal(got_q, want_q.reshape(-1, 64)), i
        rec = host(plan.recon_views[i])
        qt = O.quant_table(it.quality)
        for n, b in enumerate(idx):
            want = O.inverse_orth(O.dequantize(want_q[n], qt)) + 128
            by, bx = divmod(int(b), w // 8)
            assert np.max(np.abs(rec[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8] - want)) <= 1e-4, i
        if h * w <= 256 * 256:
            ref = O.quant_eval(img_np, qt)
            assert abs(int(sse[i]) * 2.0 ** -20 - ref["sse"]) <= nb * 2.0 ** -21 + 1e-9 * ref["sse"], i
    # Property at any size: the batch gives every plane the bits it gets alone.
    for i in rng.choice(1000, size=12, replace=False):
        s1, _, _ = R.compress_eval(imgs[i], sels[i], 1)
        assert int(host(s1)[0]) == int(sse[i]), i
    plan.close()


def test_sweep_planes_full():
    sel = R.select(R.SEL_ZIGZAG, r=1)
    for s in (0, 17, 255):
        img = synth.render(s, 512, 512, device=DEV)
        sse, _, _ = R.compress_eval(img, sel, 45)
        ref = O.retention_eval(host(img), range(1, 46))
        assert [int(v) for v in host(sse)] == [ref["sse_num"][r] for r in range(1, 46)]


@pytest.mark.parametrize("layout", ["strided", "per-plane"])
def test_sweep_batched_full(layout):
    """The sweep as the bench runs it (int32 coefficients, one launch; the
    per-plane layout with four waves per workgroup is what the autotuner picks)."""
    imgs = [synth.render(s, 512, 512, device=DEV) for s in range(256)]
    sel = R.select(R.SEL_ZIGZAG, r=1)
    tuning = R.Tuning(1, 4, 0, R.LAYOUT_STRIDED) if layout == "strided" else \
        R.Tuning(4, 1, 0, R.LAYOUT_PER_PLANE)
    plan = R.BatchPlan(imgs, [sel] * 256, R.COEF_I32, recon=False, r_count=45, tuning=tuning)
    plan.sse.fill_(-1)
    plan.run()
    sse = host(plan.sse)
    for s in range(256):
        s1, _, _ = R.compress_eval(imgs[s], sel, 45)
        assert np.array_equal(host(s1), sse[s]), s
    for s in (3, 128):
        ref = O.retention_eval(host(imgs[s]), range(1, 46))
        assert [int(v) for v in sse[s]] == [ref["sse_num"][r] for r in range(1, 46)], s
    rng = np.random.default_rng(11)
    for s in (0, 77, 255):
        idx = sample_idx(rng, 4096, 24)
        want = O.forward_blocks(O.sample_blocks(host(imgs[s]), idx), 0) * O.retention_mask(1)
        got = host(plan.coef_views[s][torch.from_numpy(idx).to(DEV)]).astype(np.int64)
        assert np.array_equal(got, want.reshape(-1, 64)), s
    plan.close()


@pytest.mark.parametrize("mode", ["sweep", "quant"])
def test_frame_error_sums_split_into_bands(frame, mode):
    """Error sums of the whole 8192 x 8192 frame (capped grid, several chunks per
    wave, one atomic per wave) equal the sums over four 2048-row bands, each
    taken alone, and the one-plane batch."""
    img, _ = frame
    if mode == "sweep":
        sel, count = R.select(R.SEL_ZIGZAG, r=1), 45
    else:
        sel, count = R.select(R.SEL_QUANT, quality=50, level_shift=128), 1
    whole, _, _ = R.compress_eval(img, sel, count)
    whole = host(whole).astype(np.int64)
    bands = sum(host(R.compress_eval(img[k * 2048:(k + 1) * 2048], sel, count)[0]).astype(np.int64)
                for k in range(4))
    assert np.array_equal(whole, bands)
    for lay in (R.LAYOUT_STRIDED, R.LAYOUT_PER_PLANE):
        # Per plane: one workgroup takes all 8192 items of the frame.
        plan = R.BatchPlan([img], [sel], None, recon=False, r_count=count,
                           tuning=R.Tuning(4, 2, 0, lay))
        plan.run()
        assert np.array_equal(host(plan.sse).reshape(-1).astype(np.int64), whole), lay
        plan.close()
    if mode == "sweep":
        assert np.all(np.diff(whole) <= 0)          # dropping fewer coefficients never adds error


def test_quality_plan_full_sampled():
    """The comparison workload as timed: one plan per transform over the 256
    planes of 512 x 512, r = 1..45.  Two sampled planes against the oracle at
    r = 1, 10, 45 (exact for the integer transforms), and the plan's rows equal
    the same planes swept alone."""
    imgs = [synth.render(s, 512, 512, device=DEV) for s in range(256)]
    nwin = 505 * 505
    quant = (16 * 16) * 2.0 ** -33 / nwin
    for t, name in ((R.T_DCT, "dct"), (R.T_RDCT, "rdct"), (R.T_SDCT, "sdct")):
        plan = R.QualityPlan(imgs, t, 1, 45)
        plan.run()
        sse, uqi = host(plan.sse).astype(np.int64), host(plan.uqi).astype(np.int64)
        for s in (5, 200):
            s1, u1 = R.quality_sweep(imgs[s], t, 1, 45)
            assert np.array_equal(host(s1).astype(np.int64), sse[s]), (name, s)
            assert np.array_equal(host(u1).astype(np.int64), uqi[s]), (name, s)
            x = host(imgs[s]).astype(np.int64)
            for r in (1, 10, 45):
                got_u = int(uqi[s, r - 1]) * 2.0 ** -32 / nwin
                if t == R.T_DCT:
                    rec = O.retention_recon(x.astype(np.uint8), name, r)
                    want = float(np.sum((x - rec) ** 2))
                    got = int(sse[s, r - 1]) * 2.0 ** -20
                    assert abs(got - want) <= 256 * 2.0 ** -21 + 1e-9 * want, (name, s, r)
                    assert abs(got_u - O.uqi(x, rec)) <= quant + 1e-9, (name, s, r)
                else:
                    num, d = O.integer_numerators(x.astype(np.uint8), name, r)
                    assert int(sse[s, r - 1]) == int(np.sum((d * x - num) ** 2)), (name, s, r)
                    want_u = float(np.mean(O.uqi_map_exact(x, num, d)))
                    assert abs(got_u - want_u) <= quant + 1e-12, (name, s, r)
        plan.close()
