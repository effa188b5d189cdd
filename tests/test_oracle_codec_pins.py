"""Pins of the codec-output oracle (CPU only): run-length coding against brute
force and hand-worked blocks, the 8-bit reconstruction against perfect
reconstruction and an independent float route."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1402_6034_amd import synth


def test_rle_hand_examples():
    assert O.rle_encode([0] * 64) == []
    assert O.rle_encode([37] + [0] * 63) == [(0, 37)]
    assert O.rle_encode([5, 0, 0, 0, 0, -2, 0, 0]) == [(0, 5), (4, -2)]
    assert O.rle_encode([0, 0, 1]) == [(2, 1)]


def test_rle_round_trip_brute_force():
    # every zero pattern of length 10 with values drawn from +-1..+-300
    rng = np.random.default_rng(0)
    for bits in itertools.product([0, 1], repeat=10):
        v = np.array(bits) * rng.integers(1, 300, size=10) * rng.choice([-1, 1], size=10)
        p = O.rle_encode(v)
        assert len(p) == int(np.count_nonzero(v))
        assert np.array_equal(O.rle_decode(p, 10), v)
        # runs + values + trailing zeros cover the sequence
        last = max([i for i in range(10) if v[i] != 0], default=-1)
        assert sum(r for r, _ in p) + len(p) == last + 1


def test_zigzag_scan_round_trip():
    blk = np.arange(64).reshape(8, 8) - 20
    for n in (1, 6, 28, 64):
        seq = O.zigzag_scan(blk, n)
        back = O.zigzag_unscan(seq)
        mask = O.retention_mask(n).astype(bool)
        assert np.array_equal(back[mask], blk[mask]) and np.all(back[~mask] == 0)
    # the scan starts (0,0), (0,1), (1,0), (2,0) (Section 3, JPEG order)
    assert list(O.zigzag_scan(blk, 4)) == [blk[0, 0], blk[0, 1], blk[1, 0], blk[2, 0]]


def test_u8_rounding_is_half_away_and_clamped():
    r = np.array([-10000, -288, -287, 0, 287, 288, 576 * 10 + 287, 576 * 10 + 288, 576 * 300])
    assert list(O.u8_from_numerator(r)) == [0, 0, 0, 0, 0, 1, 10, 11, 255]
    # the exact integer route equals the float route of Matlab's round
    rr = np.random.default_rng(1).integers(-40000, 200000, size=5000)
    rr = np.concatenate([rr, 576 * np.arange(-3, 260) + 288])
    assert np.array_equal(O.u8_from_numerator(rr), O.u8_from_float(rr / 576.0))


def test_full_retention_gives_the_original_pixels():
    img = synth.render_np(5, 40, 56)
    enc = O.codec_encode(img, "zigzag", r=64)
    assert np.array_equal(enc["recon_u8"], img)


def test_constant_plane_codes_dc_only():
    img = np.full((16, 24), 131, dtype=np.uint8)
    enc = O.codec_encode(img, "zigzag", r=10)
    assert all(p == [(0, 64 * 131)] for p in enc["pairs"])
    assert np.all(enc["recon_u8"] == 131)


@pytest.mark.parametrize("mode,kw", [("zigzag", {"r": 10}), ("zigzag", {"r": 45}),
                                     ("quant", {"quality": 50}), ("quant", {"quality": 90})])
def test_decode_recovers_the_kept_coefficients(mode, kw):
    img = synth.render_np(6, 48, 40)
    enc = O.codec_encode(img, mode, **kw)
    nby, nbx = O.n_blocks(*img.shape)
    dec = O.codec_decode_coefs(enc["pairs"], enc["n_kept"], nby, nbx)
    mask = O.retention_mask(enc["n_kept"]).astype(bool)
    assert np.array_equal(dec[..., mask], enc["coefs"][..., mask])
    assert np.all(dec[..., ~mask] == 0)
    assert np.array_equal(enc["counts"], [len(p) for p in enc["pairs"]])


def test_quant_u8_matches_the_float_reconstruction():
    img = synth.render_np(7, 32, 32)
    enc = O.codec_encode(img, "quant", quality=30)
    ref = O.quant_eval(img, O.quant_table(30))
    assert np.max(np.abs(enc["recon_float"] - ref["recon"])) < 1e-9
    assert np.array_equal(enc["recon_u8"], O.u8_from_float(ref["recon"]))
