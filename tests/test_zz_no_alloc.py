"""rdct_codec_pack_noalloc (the pack step with the library's own workspace, for
callers that cannot allocate) gives what rdct_codec_pack gives with a caller
workspace, on two calls in a row on one GPU, the second on a smaller plane (so
the array still holds the first call's prefixes), and it rejects planes beyond
its workspace."""
import numpy as np
import pytest
import torch

from paper_1402_6034_amd import synth

pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1402_6034_amd.rdct")


def _pack_noalloc(c, offsets, packed):
    return R.lib().rdct_codec_pack_noalloc(
        R._ptr(c.counts), R._ptr(c.group_pairs), R._ptr(c.slots), c.w, c.h, R._ptr(offsets),
        R._ptr(packed), packed.numel(), R._stream(None))


@pytest.mark.parametrize("sel", [R.select(R.SEL_QUANT, quality=50, level_shift=128),
                                 R.select(R.SEL_ZIGZAG, r=21)])
def test_noalloc_pack_equals_pack_twice(sel):
    for h, w, seed in ((2048, 1536, 3), (200, 136, 4)):     # 49,152 then 425 blocks
        img = torch.from_numpy(synth.render_np(seed, h, w)).cuda()
        c = R.Codec(h, w, "cuda")
        c.encode(img, sel)
        c.pack()
        offsets = torch.full_like(c.offsets, -1)
        packed = torch.full_like(c.packed, -7)
        assert _pack_noalloc(c, offsets, packed) == R.OK
        torch.cuda.synchronize()
        assert torch.equal(offsets, c.offsets), (h, w)
        total = int(c.offsets[-1])
        assert total > 0
        assert torch.equal(packed[:total], c.packed[:total]), (h, w)


def test_noalloc_pack_rejects_planes_beyond_its_workspace():
    t = torch.zeros(1024, dtype=torch.int32, device="cuda")
    # 2^22 + 1 blocks: the first plane size beyond the codec's maximum.
    st = R.lib().rdct_codec_pack_noalloc(R._ptr(t), R._ptr(t), R._ptr(t), 8 * 4097, 8 * 1024,
                                         R._ptr(t), R._ptr(t), 0, R._stream(None))
    assert st == R.ERR_UNSUPPORTED
    st = R.lib().rdct_codec_pack_noalloc(None, R._ptr(t), R._ptr(t), 64, 64, R._ptr(t), R._ptr(t),
                                         0, R._stream(None))
    assert st == R.ERR_INVALID_ARG
