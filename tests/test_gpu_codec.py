"""Codec output (rdct_codec_encode / rdct_codec_pack) against the oracle.

Bars: run-length pairs, counts, offsets and the keep-r 8-bit reconstruction
bit-exact (integer work, the rounding decided exactly through the numerator);
the quantisation path's 8-bit pixels equal except where the float64
reconstruction lies within 1e-9 of a rounding boundary (both sides round in
float64, in different operation orders).
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


def run_codec(img, sel):
    h, w = img.shape
    c = R.Codec(h, w, DEV)
    c.encode(g(img), sel)
    c.pack()
    torch.cuda.synchronize()
    return c


def check_pairs(c, enc):
    counts = c.counts.cpu().numpy().astype(np.int64) & 0xffff
    assert np.array_equal(counts, enc["counts"])
    off = c.offsets.cpu().numpy().astype(np.int64)
    assert off[0] == 0 and np.array_equal(np.diff(off), enc["counts"])
    assert c.pairs_host() == [list(p) for p in enc["pairs"]]


SHAPES = [(8, 8), (40, 56), (13, 21), (64, 200), (72, 72)]


@pytest.mark.parametrize("h,w", SHAPES)
@pytest.mark.parametrize("r", [1, 10, 45, 64])
def test_zigzag_codec(h, w, r):
    img = synth.render_np(h * 7 + w + r, h, w)
    enc = O.codec_encode(img, "zigzag", r=r)
    c = run_codec(img, R.select(R.SEL_ZIGZAG, r=r))
    check_pairs(c, enc)
    assert np.array_equal(c.recon.cpu().numpy(), enc["recon_u8"])
    if r == 64:
        assert np.array_equal(c.recon.cpu().numpy(), img)


@pytest.mark.parametrize("h,w", SHAPES)
@pytest.mark.parametrize("quality", [1, 10, 50, 90, 100])
def test_quant_codec(h, w, quality):
    img = synth.render_np(h + w + quality, h, w)
    enc = O.codec_encode(img, "quant", quality=quality, level_shift=128)
    c = run_codec(img, R.select(R.SEL_QUANT, quality=quality, level_shift=128))
    check_pairs(c, enc)
    got = c.recon.cpu().numpy()
    a = enc["recon_float"]
    near = np.abs(np.abs(a - np.floor(a)) - 0.5) < 1e-9
    assert np.array_equal(got[~near], enc["recon_u8"][~near])


def test_quant_codec_dense_groups():
    """Uniform noise at quality 100: nearly every coefficient survives, so the
    first 64-block group fills its slot almost to the 4096 pairs it holds, and
    every wave takes the reconstruction's dense path (more than 10 nonzero
    positions)."""
    img = np.random.default_rng(5).integers(0, 256, size=(64, 136), dtype=np.uint8)
    enc = O.codec_encode(img, "quant", quality=100, level_shift=128)
    assert int(np.sum(enc["counts"][:64])) > 4000
    c = run_codec(img, R.select(R.SEL_QUANT, quality=100, level_shift=128))
    check_pairs(c, enc)
    got = c.recon.cpu().numpy()
    a = enc["recon_float"]
    near = np.abs(np.abs(a - np.floor(a)) - 0.5) < 1e-9
    assert np.array_equal(got[~near], enc["recon_u8"][~near])


def test_pack_respects_capacity_and_pitched_output():
    img = synth.render_np(3, 48, 80)
    h, w = img.shape
    enc = O.codec_encode(img, "zigzag", r=20)
    c = R.Codec(h, w, DEV)
    buf = torch.full((h, w + 5), 7, dtype=torch.uint8, device=DEV)
    c.recon = buf[:, :w]                      # 85-byte rows: not 8-byte aligned
    c.encode(g(img), R.select(R.SEL_ZIGZAG, r=20))
    total = int(enc["counts"].sum())
    cap = total // 2
    c.packed.fill_(-1)
    L = R.lib()
    st = L.rdct_codec_pack(c.counts.data_ptr(), c.group_pairs.data_ptr(), c.slots.data_ptr(), w, h,
                           c.offsets.data_ptr(), c.packed.data_ptr(), cap,
                           c.workspace.data_ptr(), None)
    assert st == R.OK
    torch.cuda.synchronize()
    assert int(c.offsets[-1]) == total
    packed = c.packed.cpu().numpy()
    assert np.all(packed[cap:] == -1) and np.all(packed[:cap] != -1) if cap < total else True
    assert np.array_equal(buf[:, :w].cpu().numpy(), enc["recon_u8"])
    assert np.all(buf[:, w:].cpu().numpy() == 7)


def test_encode_without_reconstruction():
    img = synth.render_np(4, 32, 64)
    h, w = img.shape
    c = R.Codec(h, w, DEV)
    c.recon.fill_(9)
    c.encode(g(img), R.select(R.SEL_QUANT, quality=60, level_shift=128), recon=False)
    c.pack()
    check_pairs(c, O.codec_encode(img, "quant", quality=60))
    assert torch.all(c.recon == 9)
