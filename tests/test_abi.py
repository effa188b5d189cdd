"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/*.h declares, and rejects bad arguments before launching anything."""
import ctypes
import glob
import os
import re

import pytest
import torch

from conftest import ROOT

R = pytest.importorskip("paper_1402_6034_amd.rdct")


def _declared_symbols():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        for m in re.finditer(r"\b(rdct_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_core_path():
    names = _declared_symbols()
    for n in ("rdct_forward", "rdct_inverse", "rdct_compress_eval", "rdct_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = R.lib()
    missing = [n for n in _declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_units():
    assert R.lib().rdct_status_string(R.ERR_INVALID_ARG).decode() == "invalid argument"
    assert R.rdct_sse_unit(R.SEL_ZIGZAG) == 1.0 / 576 ** 2
    assert R.rdct_sse_unit(R.SEL_QUANT) == 2.0 ** -20
    assert R.rdct_psnr(0, R.SEL_ZIGZAG, 8, 8) == float("inf")
    # sse = 576^2 * 64 * 255^2 over an 8x8 plane: MSE = 255^2 -> 0 dB.
    assert abs(R.rdct_psnr(576 ** 2 * 64 * 255 ** 2, R.SEL_ZIGZAG, 8, 8)) < 1e-12
    assert R.rdct_num_blocks(9, 17) == 2 * 3
    assert R.rdct_num_blocks(0, 5) == 0


# Fake, never-dereferenced addresses: every case below must be rejected during
# validation.  Skipped when a GPU is present so that a validation bug could never
# turn into a launch on a fake pointer.
needs_no_gpu = pytest.mark.skipif(torch.cuda.is_available(), reason="host-only validation checks")
FAKE_SRC, FAKE_DST, FAKE_SSE = 1 << 20, 1 << 21, 1 << 22


def _fwd(src, w, h, pitch, sel, coef, ctype):
    return R.lib().rdct_forward(src, w, h, pitch, ctypes.byref(sel), coef, ctype, None)


@needs_no_gpu
@pytest.mark.parametrize("case", [
    dict(src=None), dict(w=0), dict(h=-1), dict(pitch=7), dict(coef=None),
    dict(coef=FAKE_DST + 4), dict(ctype=9), dict(sel=R.select(R.SEL_ZIGZAG, r=0)),
    dict(sel=R.select(R.SEL_ZIGZAG, r=65)), dict(sel=R.select(R.SEL_QUANT, quality=0)),
    dict(sel=R.select(R.SEL_QUANT, quality=101)), dict(sel=R.select(R.SEL_QUANT, qtable=[0] * 64)),
    dict(sel=R.select(R.SEL_QUANT, quality=50), ctype=R.COEF_F32),
    dict(sel=R.select(R.SEL_NONE, level_shift=256)), dict(sel=R.select(7)),
])
def test_forward_rejects(case):
    a = dict(src=FAKE_SRC, w=16, h=16, pitch=16, sel=R.select(R.SEL_NONE), coef=FAKE_DST,
             ctype=R.COEF_I32)
    a.update(case)
    assert _fwd(a["src"], a["w"], a["h"], a["pitch"], a["sel"], a["coef"], a["ctype"]) == R.ERR_INVALID_ARG


@needs_no_gpu
def test_forward_rejects_huge_plane_as_unsupported():
    assert _fwd(FAKE_SRC, 70000, 70000, 70000, R.select(R.SEL_NONE), FAKE_DST,
                R.COEF_I32) == R.ERR_UNSUPPORTED


def _eval(sel, r_count=1, w=64, h=64, sse=FAKE_SSE, coef=None, ctype=R.COEF_I32, recon=None,
          rpitch=0):
    return R.lib().rdct_compress_eval(FAKE_SRC, w, h, w, ctypes.byref(sel), r_count, coef, ctype,
                                      recon, rpitch, sse, None)


@needs_no_gpu
def test_compress_eval_rejects():
    z = R.select(R.SEL_ZIGZAG, r=20)
    q = R.select(R.SEL_QUANT, quality=50, level_shift=128)
    assert _eval(z, sse=None) == R.ERR_INVALID_ARG
    assert _eval(z, r_count=0) == R.ERR_INVALID_ARG
    assert _eval(z, r_count=46) == R.ERR_INVALID_ARG          # r up to 65
    assert _eval(q, r_count=2) == R.ERR_INVALID_ARG
    assert _eval(R.select(R.SEL_NONE), r_count=2) == R.ERR_INVALID_ARG
    assert _eval(z, recon=FAKE_DST, rpitch=10) == R.ERR_INVALID_ARG
    assert _eval(q, coef=FAKE_DST, ctype=R.COEF_F32) == R.ERR_INVALID_ARG
    assert _eval(z, r_count=2, w=60) == R.ERR_UNSUPPORTED     # sweep needs whole blocks
    assert _eval(z, w=24000, h=20000) == R.ERR_UNSUPPORTED    # 7.5 M blocks: beyond the SSE range


@needs_no_gpu
def test_inverse_rejects():
    L = R.lib()
    sel = R.select(R.SEL_ZIGZAG, r=10)
    assert L.rdct_inverse(None, R.COEF_I32, 8, 8, ctypes.byref(sel), FAKE_DST, 8, None) == R.ERR_INVALID_ARG
    assert L.rdct_inverse(FAKE_SRC, R.COEF_I32, 8, 8, ctypes.byref(sel), FAKE_DST, 4, None) == R.ERR_INVALID_ARG
    qs = R.select(R.SEL_QUANT, quality=50)
    assert L.rdct_inverse(FAKE_SRC, R.COEF_F32, 8, 8, ctypes.byref(qs), FAKE_DST, 8, None) == R.ERR_INVALID_ARG


@needs_no_gpu
def test_batch_plan_create_rejects():
    L = R.lib()
    h = ctypes.c_void_p()

    def desc(mode, **kw):
        d = R.PlaneDesc()
        d.src, d.width, d.height, d.src_pitch = FAKE_SRC, 64, 64, 64
        d.sel = R.select(mode, r=10, quality=50)
        for k, v in kw.items():
            setattr(d, k, v)
        return d
    arr = (R.PlaneDesc * 2)(desc(R.SEL_QUANT), desc(R.SEL_ZIGZAG))
    assert L.rdct_batch_plan_create(arr, 2, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    arr = (R.PlaneDesc * 2)(desc(R.SEL_QUANT), desc(R.SEL_QUANT, coef_out=FAKE_DST))
    assert L.rdct_batch_plan_create(arr, 2, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    arr = (R.PlaneDesc * 1)(desc(R.SEL_QUANT, width=0))
    assert L.rdct_batch_plan_create(arr, 1, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    arr = (R.PlaneDesc * 1)(desc(R.SEL_QUANT))
    assert L.rdct_batch_plan_create(arr, 1, R.COEF_I16, None, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    assert L.rdct_batch_plan_create(arr, 0, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    assert L.rdct_batch_run(None, None) == R.ERR_INVALID_ARG
    assert L.rdct_batch_autotune(None, 3, None, None) == R.ERR_INVALID_ARG
    # Sweeps: zig-zag only, r range within 64, whole blocks, r_count >= 1.
    sw = L.rdct_batch_plan_create_sweep
    arr = (R.PlaneDesc * 1)(desc(R.SEL_QUANT))
    assert sw(arr, 1, 4, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    arr = (R.PlaneDesc * 1)(desc(R.SEL_ZIGZAG))
    assert sw(arr, 1, 0, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    assert sw(arr, 1, 56, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG
    arr = (R.PlaneDesc * 1)(desc(R.SEL_ZIGZAG, width=60))
    assert sw(arr, 1, 4, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_UNSUPPORTED
    arr = (R.PlaneDesc * 1)(desc(R.SEL_NONE))
    assert sw(arr, 1, 2, R.COEF_I16, FAKE_SSE, None, ctypes.byref(h)) == R.ERR_INVALID_ARG


def test_quality_units_and_windows():
    assert R.rdct_quality_sse_unit(R.T_RDCT) == 1.0 / 576 ** 2
    assert R.rdct_quality_sse_unit(R.T_SDCT) == 1.0 / 64 ** 2
    assert R.rdct_quality_sse_unit(R.T_DCT) == 2.0 ** -20
    assert R.rdct_quality_sse_unit(R.T_RDCT_CEIL) == 2.0 ** -20
    assert R.rdct_quality_sse_unit(9) == 0.0
    assert R.rdct_quality_windows(512, 512) == 505 * 505
    assert R.rdct_quality_windows(8, 16) == 9
    assert R.rdct_quality_windows(7, 100) == 0


@needs_no_gpu
def test_quality_sweep_rejects():
    L = R.lib()

    def call(w=64, h=64, pitch=64, t=R.T_RDCT, r0=1, n=45, sse=FAKE_SSE, uqi=FAKE_DST, src=FAKE_SRC):
        return L.rdct_quality_sweep(src, w, h, pitch, t, r0, n, sse, uqi, None)
    assert call(src=None) == R.ERR_INVALID_ARG
    assert call(sse=None) == R.ERR_INVALID_ARG
    assert call(uqi=FAKE_DST + 4) == R.ERR_INVALID_ARG
    assert call(t=9) == R.ERR_INVALID_ARG
    assert call(r0=0) == R.ERR_INVALID_ARG
    assert call(r0=20, n=46) == R.ERR_INVALID_ARG
    assert call(n=0) == R.ERR_INVALID_ARG
    assert call(pitch=63) == R.ERR_INVALID_ARG
    assert call(t=R.T_RDCT_FLOOR) == R.ERR_UNSUPPORTED      # floor(2C): singular
    assert call(w=60) == R.ERR_UNSUPPORTED                   # needs whole blocks
    assert call(w=8192, h=8200, pitch=8192) == R.ERR_UNSUPPORTED  # above 2^20 blocks
    h = ctypes.c_void_p()
    d = (R.QualityDesc * 2)()
    for x in d:
        x.src, x.width, x.height, x.src_pitch = FAKE_SRC, 64, 64, 64
    d[1].width = 12
    assert L.rdct_quality_plan_create(d, 2, R.T_DCT, 1, 45, FAKE_SSE, FAKE_DST, ctypes.byref(h)) == R.ERR_UNSUPPORTED
    d[1].width = 64
    assert L.rdct_quality_plan_create(d, 2, R.T_RDCT_FLOOR, 1, 45, FAKE_SSE, FAKE_DST, ctypes.byref(h)) == R.ERR_UNSUPPORTED
    assert L.rdct_quality_plan_create(d, 0, R.T_DCT, 1, 45, FAKE_SSE, FAKE_DST, ctypes.byref(h)) == R.ERR_INVALID_ARG
    assert L.rdct_quality_plan_run(None, None) == R.ERR_INVALID_ARG


@needs_no_gpu
def test_codec_rejects():
    L = R.lib()
    z = R.select(R.SEL_ZIGZAG, r=10)

    def enc(sel=z, w=64, h=64, counts=FAKE_DST, gp=FAKE_DST, slots=FAKE_DST, recon=None, rp=0):
        return L.rdct_codec_encode(FAKE_SRC, w, h, w, ctypes.byref(sel), counts, gp, slots, recon,
                                   rp, None)
    assert enc(sel=R.select(R.SEL_ZIGZAG, r=0)) == R.ERR_INVALID_ARG
    assert enc(counts=None) == R.ERR_INVALID_ARG
    assert enc(slots=FAKE_DST + 2) == R.ERR_INVALID_ARG
    assert enc(recon=FAKE_DST, rp=10) == R.ERR_INVALID_ARG
    assert enc(w=20000, h=16400) == R.ERR_UNSUPPORTED        # above 2^22 blocks
    assert L.rdct_codec_pack(FAKE_DST, FAKE_DST, FAKE_DST, 64, 64, None, FAKE_DST, 10, FAKE_DST,
                             None) == R.ERR_INVALID_ARG
    assert L.rdct_codec_pack(FAKE_DST, FAKE_DST, FAKE_DST, 64, 64, FAKE_DST, None, 10, FAKE_DST,
                             None) == R.ERR_INVALID_ARG
    assert R.rdct_codec_groups(64, 64) == 1 and R.rdct_codec_groups(72, 64) == 2


def test_psnr_of_many_planes_matches_single_calls():
    import numpy as np
    rng = np.random.default_rng(3)
    widths, heights = [8, 64, 13], [8, 40, 21]
    sse = rng.integers(0, 2 ** 40, size=(3, 5)).astype(np.uint64)
    sse[1, 2] = 0
    for mode in (R.SEL_ZIGZAG, R.SEL_QUANT):
        ps, mean = R.rdct_psnr_planes(sse, 5, mode, widths, heights, mean=True)
        for i in range(3):
            for j in range(5):
                assert ps[i, j] == R.rdct_psnr(int(sse[i, j]), mode, widths[i], heights[i])
        assert np.isinf(mean[2])
        assert abs(mean[0] - ps[:, 0].mean()) < 1e-12
    with pytest.raises(RuntimeError):
        R.rdct_psnr_planes(sse, 5, R.SEL_ZIGZAG, [8, 0, 8], heights)


def test_quality_metrics_units():
    import numpy as np
    sse = np.array([576 ** 2 * 64, 0], dtype=np.uint64)
    uqi = np.array([2 ** 32, 2 ** 31], dtype=np.int64)
    mse, mu = R.rdct_quality_metrics(sse, uqi, R.T_RDCT, 8, 8)
    assert mse.tolist() == [1.0, 0.0] and mu.tolist() == [1.0, 0.5]
    mse, mu = R.rdct_quality_metrics(np.array([2 ** 20 * 9]), np.array([2 ** 32 * 4]), R.T_DCT, 9, 9)
    assert mse[0] == 1.0 / 9 and mu[0] == 1.0
    with pytest.raises(RuntimeError):
        R.rdct_quality_metrics(sse, uqi, R.T_RDCT_FLOOR, 8, 8)


def test_pair_words_decode():
    import numpy as np
    words = np.array([(5 << 16) | 0xfffe, (63 << 16) | 0x7fff, 0x8000, 0], dtype=np.uint32).view(np.int32)
    runs, vals = R.rdct_codec_unpack_pairs(words)
    assert runs.tolist() == [5, 63, 0, 0] and vals.tolist() == [-2, 32767, -32768, 0]


def test_set_tuning_rejects_a_null_plan_and_invalid_geometry():
    t = R.Tuning(1, 4, 0, R.LAYOUT_STRIDED, 0)
    assert R.lib().rdct_batch_plan_set_tuning(None, ctypes.byref(t)) == R.ERR_INVALID_ARG


@needs_no_gpu
def test_device_psnr_rejects_bad_arguments():
    L = R.lib()
    assert L.rdct_psnr_device(None, 3, 1, R.SEL_ZIGZAG, None, None, None, None) == R.ERR_INVALID_ARG
    assert L.rdct_psnr_device(1 << 20, 3, 0, R.SEL_ZIGZAG, 1 << 21, 1 << 22, None, None) == R.ERR_INVALID_ARG
    assert L.rdct_psnr_device(1 << 20, 3, 1, 7, 1 << 21, 1 << 22, None, None) == R.ERR_INVALID_ARG
    assert L.rdct_psnr_device(1 << 20 | 4, 3, 1, R.SEL_ZIGZAG, 1 << 21, 1 << 22, None,
                              None) == R.ERR_INVALID_ARG
