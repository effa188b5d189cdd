"""Seeded random cases against the oracle: sizes (ragged, not multiples of 8),
selections (r, quality, level shift) and transforms drawn from a seeded
generator per case, each case through the fused evaluation, the codec and, for sides that are
multiples of 8, the comparison path.  Bars as in the dedicated tests: integer
results bit-exact, float32 reconstructions within 1e-4, the quantisation SSE
within the per-block fixed-point step, 8-bit quantisation pixels equal away
from rounding ties, comparison sums exact for the integer transforms.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1402_6034_amd import synth

pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1402_6034_amd.rdct")
DEV = "cuda:0"


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def case_plane(seed):
    """A generator for the case's other draws, and its plane (sides 1..96)."""
    rng = np.random.default_rng(seed)
    h, w = int(rng.integers(1, 97)), int(rng.integers(1, 97))
    return rng, h, w, synth.render_np(int(rng.integers(0, 1 << 30)), h, w)


@pytest.mark.parametrize("case", range(12))
def test_random_retention(case):
    rng, h, w, img = case_plane(1010 + case)
    r = int(rng.integers(1, 65))
    ref = O.retention_eval(img, [r], recon_r=r)
    sse, coef, rec = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=r), 1, R.COEF_I32, True)
    assert int(host(sse)[0]) == ref["sse_num"][r], (h, w, r)
    assert np.array_equal(host(coef).astype(np.int64).reshape(-1, 64),
                          (ref["Y"] * O.retention_mask(r)).reshape(-1, 64)), (h, w, r)
    assert np.max(np.abs(host(rec) - ref["recon"])) <= 1e-4, (h, w, r)
    enc = O.codec_encode(img, "zigzag", r=r)
    c = R.Codec(h, w, DEV)
    c.encode(g(img), R.select(R.SEL_ZIGZAG, r=r))
    c.pack()
    assert c.pairs_host() == [list(p) for p in enc["pairs"]], (h, w, r)
    assert np.array_equal(host(c.recon), enc["recon_u8"]), (h, w, r)


@pytest.mark.parametrize("case", range(12))
def test_random_quantisation(case):
    rng, h, w, img = case_plane(2020 + case)
    quality = int(rng.integers(1, 101))
    shift = int(rng.choice([0, 128, int(rng.integers(0, 256))]))
    qt = O.quant_table(quality)
    ref = O.quant_eval(img, qt, level_shift=shift)
    sel = R.select(R.SEL_QUANT, quality=quality, level_shift=shift)
    sse, q, rec = R.compress_eval(g(img), sel, 1, R.COEF_I16, True)
    nb = ((h + 7) // 8) * ((w + 7) // 8)
    assert np.array_equal(host(q).astype(np.int64).reshape(-1, 64),
                          ref["q"].reshape(-1, 64)), (h, w, quality, shift)
    assert np.max(np.abs(host(rec) - ref["recon"])) <= 1e-4, (h, w, quality, shift)
    assert abs(int(host(sse)[0]) * 2.0 ** -20 - ref["sse"]) <= nb * 2.0 ** -21 + 1e-9 * ref["sse"]
    enc = O.codec_encode(img, "quant", quality=quality, level_shift=shift)
    c = R.Codec(h, w, DEV)
    c.encode(g(img), sel)
    c.pack()
    assert c.pairs_host() == [list(p) for p in enc["pairs"]], (h, w, quality, shift)
    f = enc["recon_float"]
    near = np.abs(np.abs(f - np.floor(f)) - 0.5) < 1e-9
    assert np.array_equal(host(c.recon)[~near], enc["recon_u8"][~near]), (h, w, quality, shift)


@pytest.mark.parametrize("case", range(8))
def test_random_comparison_integer_transforms(case):
    rng = np.random.default_rng(303 + case)
    h, w = 8 * int(rng.integers(1, 13)), 8 * int(rng.integers(1, 13))
    img = synth.render_np(int(rng.integers(0, 1 << 30)), h, w)
    t, name = [(R.T_RDCT, "rdct"), (R.T_SDCT, "sdct")][case % 2]
    r0 = int(rng.integers(1, 60))
    count = int(rng.integers(1, 66 - r0))
    sse, uqi = R.quality_sweep(g(img), t, r0, count)
    sse, uqi = host(sse).astype(np.int64), host(uqi).astype(np.int64)
    x = img.astype(np.int64)
    nwin = max(1, (h - 7) * (w - 7))
    tiles = -(-h // 32) * -(-w // 32)
    for i, r in enumerate(range(r0, r0 + count)):
        num, d = O.integer_numerators(img, name, r)
        assert int(sse[i]) == int(np.sum((d * x - num) ** 2)), (h, w, name, r)
        if h >= 8 and w >= 8:
            want = float(np.mean(O.uqi_map_exact(x, num, d)))
            assert abs(int(uqi[i]) * 2.0 ** -32 / nwin - want) <= tiles * 2.0 ** -33 / nwin + 1e-12
