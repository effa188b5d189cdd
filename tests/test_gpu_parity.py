"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bars: integer coefficients and quantised values bit-exact; exact integer SSE
equal; float32 scaled coefficients and reconstructions within 1e-4 of the
float64 oracle; PSNR within 1e-3 dB.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1402_6034_amd import synth

pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1402_6034_amd.rdct")
DEV = "cuda:0"
TOL = 1e-4
PSNR_TOL = 1e-3


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def flat(blocks):
    return np.asarray(blocks).reshape(-1, 64)


def pitched(img, extra):
    """Device plane whose rows are `extra` bytes longer than its width."""
    h, w = img.shape
    buf = torch.zeros((h, w + extra), dtype=torch.uint8, device=DEV)
    buf[:, :w] = g(img)
    return buf[:, :w]


def sign_pattern_plane():
    """64 blocks; block (k, l) is 255 where C0[k,i] C0[l,j] > 0, else 0, so it
    reaches the largest |Y_kl|.  Plus constant, checkerboard and ramp blocks."""
    c0 = O.round_off_matrix()
    tiles = [255 * (np.outer(c0[k], c0[l]) > 0) for k in range(8) for l in range(8)]
    tiles += [np.zeros((8, 8)), np.full((8, 8), 255), 255 * (np.indices((8, 8)).sum(0) % 2),
              np.tile(np.arange(8) * 36, (8, 1)), np.full((8, 8), 129), np.full((8, 8), 127),
              255 * (np.outer(c0[7], c0[7]) < 0), 255 * (np.outer(c0[1], c0[5]) < 0)]
    rows = [np.concatenate(tiles[i:i + 8], axis=1) for i in range(0, 72, 8)]
    return np.concatenate(rows, axis=0).astype(np.uint8)


SHAPES = [(8, 8), (8, 64), (64, 8), (16, 200), (24, 1032), (13, 21), (1, 1), (7, 9), (520, 8),
          (512, 512)]


def plane(h, w, seed=0):
    return synth.render_np(seed, h, w)


# ---------------------------------------------------------------------------
# Forward
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("h,w", SHAPES)
def test_forward_integer_bit_exact(h, w):
    img = plane(h, w, seed=h * 1000 + w)
    want = flat(O.forward_image(img))
    for ct in (R.COEF_I32, R.COEF_I16):
        got = host(R.forward(g(img), R.select(R.SEL_NONE), ct)).astype(np.int64)
        assert np.array_equal(got, want), ct


@pytest.mark.parametrize("extra", [8, 3, 64])
def test_forward_pitched_planes(extra):
    img = plane(40, 72, seed=extra)
    got = host(R.forward(pitched(img, extra), R.select(R.SEL_NONE), R.COEF_I32))
    assert np.array_equal(got, flat(O.forward_image(img)))


def test_forward_extreme_blocks():
    img = sign_pattern_plane()
    got = host(R.forward(g(img), R.select(R.SEL_NONE), R.COEF_I32))
    want = flat(O.forward_image(img))
    assert np.array_equal(got, want)
    assert np.abs(want).max() == 16320


@pytest.mark.parametrize("r", [1, 5, 10, 15, 45, 64])
def test_forward_retention(r):
    img = plane(64, 96, seed=r)
    y = O.forward_image(img)
    m = O.retention_mask(r)
    got = host(R.forward(g(img), R.select(R.SEL_ZIGZAG, r=r), R.COEF_I32))
    assert np.array_equal(got, flat(y * m))
    z = host(R.forward(g(img), R.select(R.SEL_ZIGZAG, r=r), R.COEF_F32))
    want = flat(O.scale_coeffs(y) * m)
    assert np.max(np.abs(z - want)) <= TOL
    assert np.all(z[:, m.reshape(-1) == 0] == 0)


@pytest.mark.parametrize("quality,shift", [(50, 128), (10, 128), (90, 128), (1, 128),
                                           (100, 128), (75, 0), (37, 128)])
def test_forward_quant_bit_exact(quality, shift):
    img = np.concatenate([plane(64, 64, seed=quality), sign_pattern_plane()], axis=0)
    qt = O.quant_table(quality)
    want = flat(O.quantize(O.forward_image(img, shift), qt))
    for ct in (R.COEF_I16, R.COEF_I32):
        got = host(R.forward(g(img), R.select(R.SEL_QUANT, quality=quality, level_shift=shift), ct))
        assert np.array_equal(got.astype(np.int64), want), ct


@pytest.mark.parametrize("qv", [1, 2, 3, 5, 6, 7])
def test_forward_quant_ties(qv):
    # Small uniform tables make exact ties z / Q = n + 1/2 frequent at the
    # positions where s_k s_l is rational.
    img = plane(96, 96, seed=qv)
    qt = np.full((8, 8), qv)
    y = O.forward_image(img, 128)
    g_ = np.diag(O.gram())
    rational = np.equal.outer(g_, g_)
    den = np.where(rational, g_[:, None] * qv, 1) * np.ones((8, 8), dtype=np.int64)
    num = 2 * np.abs(y)
    ties = rational & (num % den == 0) & ((num // den) % 2 == 1)
    want = flat(O.quantize(y, qt))
    got = host(R.forward(g(img), R.select(R.SEL_QUANT, qtable=qt.reshape(-1), level_shift=128),
                         R.COEF_I32))
    assert np.array_equal(got.astype(np.int64), want)
    assert ties.sum() > 0


# ---------------------------------------------------------------------------
# Inverse
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("h,w", [(64, 64), (13, 21), (8, 200)])
@pytest.mark.parametrize("r", [1, 10, 64])
def test_inverse_integer_path(h, w, r):
    img = plane(h, w, seed=r + h)
    y = O.forward_image(img)
    res = O.retention_eval(img, [r], recon_r=r)
    coef = g(flat(y).astype(np.int32))
    got = host(R.inverse(coef, h, w, R.select(R.SEL_ZIGZAG, r=r), R.COEF_I32))
    assert np.max(np.abs(got - res["recon"])) <= TOL
    coef16 = g(flat(y).astype(np.int16))
    got16 = host(R.inverse(coef16, h, w, R.select(R.SEL_ZIGZAG, r=r), R.COEF_I16))
    assert np.array_equal(got16, got)


def test_inverse_scaled_float_path():
    img = plane(48, 80, seed=3)
    y = O.forward_image(img)
    z = (O.scale_coeffs(y) * O.retention_mask(10)).astype(np.float32)
    got = host(R.inverse(g(flat(z)), 48, 80, R.select(R.SEL_ZIGZAG, r=10), R.COEF_F32))
    want = O.untile(O.inverse_orth(z.astype(np.float64)), 48, 80)
    assert np.max(np.abs(got - want)) <= TOL


@pytest.mark.parametrize("quality", [10, 50, 90])
def test_inverse_quant_path(quality):
    img = plane(40, 56, seed=quality)
    qt = O.quant_table(quality)
    res = O.quant_eval(img, qt)
    q = flat(res["q"])
    sel = R.select(R.SEL_QUANT, quality=quality, level_shift=128)
    for ct, dt in ((R.COEF_I16, np.int16), (R.COEF_I32, np.int32)):
        got = host(R.inverse(g(q.astype(dt)), 40, 56, sel, ct))
        assert np.max(np.abs(got - res["recon"])) <= TOL


# ---------------------------------------------------------------------------
# Fused compress + evaluate
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("h,w", [(512, 512), (13, 21), (40, 1000), (8, 8), (71, 64)])
@pytest.mark.parametrize("r", [1, 10, 45])
def test_compress_eval_retention(h, w, r):
    img = plane(h, w, seed=7 * r + w)
    res = O.retention_eval(img, [r], recon_r=r)
    sse, coef, rec = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=r), 1, R.COEF_F32, True)
    s = int(host(sse)[0])
    assert s == res["sse_num"][r]
    assert np.max(np.abs(host(rec) - res["recon"])) <= TOL
    assert np.max(np.abs(host(coef) - flat(res["Z"]))) <= TOL
    p = R.psnr_from_sse(s, R.SEL_ZIGZAG, h, w)
    if math.isfinite(res["psnr"][r]):
        assert abs(p - res["psnr"][r]) <= PSNR_TOL
    # Integer coefficient output of the same call path.
    _, c32, _ = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=r), 1, R.COEF_I32)
    assert np.array_equal(host(c32), flat(res["Y"] * O.retention_mask(r)))


@pytest.mark.parametrize("r0,count", [(1, 45), (1, 64), (5, 20), (64, 1), (3, 2)])
def test_compress_eval_sweep(r0, count):
    img = plane(128, 192, seed=r0 + count)
    rs = list(range(r0, r0 + count))
    res = O.retention_eval(img, rs)
    sse, _, _ = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=r0), count)
    got = host(sse)
    assert [int(v) for v in got] == [res["sse_num"][r] for r in rs]


def test_compress_eval_sweep_with_recon_matches_single():
    img = plane(64, 64, seed=11)
    sse, coef, rec = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=6), 10, R.COEF_I32, True)
    s1, c1, r1 = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=6), 1, R.COEF_I32, True)
    assert int(host(sse)[0]) == int(host(s1)[0])
    assert np.array_equal(host(coef), host(c1))
    assert np.array_equal(host(rec), host(r1))


@pytest.mark.parametrize("h,w,quality", [(512, 512, 50), (64, 96, 10), (64, 96, 90),
                                         (13, 21, 50), (40, 57, 75), (8, 8, 1)])
def test_compress_eval_quant(h, w, quality):
    img = plane(h, w, seed=quality + h)
    qt = O.quant_table(quality)
    res = O.quant_eval(img, qt)
    sel = R.select(R.SEL_QUANT, quality=quality, level_shift=128)
    sse, q, rec = R.compress_eval(g(img), sel, 1, R.COEF_I16, True)
    assert np.array_equal(host(q).astype(np.int64), flat(res["q"]))
    assert np.max(np.abs(host(rec) - res["recon"])) <= TOL
    nb = O.n_blocks(h, w)[0] * O.n_blocks(h, w)[1]
    got = int(host(sse)[0]) * 2.0 ** -20
    assert abs(got - res["sse"]) <= nb * 2.0 ** -21 + 1e-9 * res["sse"]
    p = R.psnr_from_sse(int(host(sse)[0]), R.SEL_QUANT, h, w)
    assert abs(p - res["psnr"]) <= PSNR_TOL
    # Without outputs: same error sum.
    s2, _, _ = R.compress_eval(g(img), sel, 1)
    assert int(host(s2)[0]) == int(host(sse)[0])


# Planes of at most 32768 blocks run in chunks of 64 blocks per wave (the high
# block of every pair empty), larger ones in chunks of 128: both sides of that
# rule, with whole and partial blocks.
@pytest.mark.parametrize("h,w", [(1024, 2048), (1032, 2048), (1021, 2047), (1025, 2041)])
def test_compress_eval_on_both_sides_of_the_chunk_rule(h, w):
    img = plane(h, w, seed=h + w)
    res = O.retention_eval(img, [10], recon_r=10)
    sse, c32, rec = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=10), 1, R.COEF_I32, True)
    assert int(host(sse)[0]) == res["sse_num"][10]
    assert np.array_equal(host(c32), flat(res["Y"] * O.retention_mask(10)))
    assert np.max(np.abs(host(rec) - res["recon"])) <= TOL
    qt = O.quant_table(50)
    qres = O.quant_eval(img, qt)
    sel = R.select(R.SEL_QUANT, quality=50, level_shift=128)
    sse, q, rec = R.compress_eval(g(img), sel, 1, R.COEF_I16, True)
    assert np.array_equal(host(q).astype(np.int64), flat(qres["q"]))
    assert np.max(np.abs(host(rec) - qres["recon"])) <= TOL
    p = R.psnr_from_sse(int(host(sse)[0]), R.SEL_QUANT, h, w)
    assert abs(p - qres["psnr"]) <= PSNR_TOL


@pytest.mark.parametrize("pitch_extra,offset", [(8, 0), (3, 1), (0, 2)])
def test_compress_eval_quant_recon_layouts(pitch_extra, offset):
    # Whole-block plane (reconstruction staged through LDS), a short last chunk
    # (200 blocks = 128 + 72), and reconstruction rows that are 16-byte aligned
    # or not; the padding around the plane must stay untouched.
    h, w = 64, 200
    img = plane(h, w, seed=5)
    res = O.quant_eval(img, O.quant_table(40))
    sel = R.select(R.SEL_QUANT, quality=40, level_shift=128)
    pitch = w + pitch_extra
    buf = torch.full((h * pitch + offset + 16,), -12345.0, dtype=torch.float32, device=DEV)
    view = buf[offset:offset + h * pitch].view(h, pitch)[:, :w]
    sse, q, rec = R.compress_eval(g(img), sel, 1, R.COEF_I16, True, recon_out=view)
    assert np.array_equal(host(q).astype(np.int64), flat(res["q"]))
    assert np.max(np.abs(host(view) - res["recon"])) <= TOL
    full = host(buf)
    mask = np.ones(full.shape, dtype=bool)
    idx = offset + np.arange(h)[:, None] * pitch + np.arange(w)[None, :]
    mask[idx.ravel()] = False
    assert np.all(full[mask] == -12345.0)


def test_constant_plane_has_zero_retention_error():
    img = np.full((64, 64), 93, dtype=np.uint8)
    sse, _, _ = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=1), 45)
    assert np.all(host(sse) == 0)


# ---------------------------------------------------------------------------
# Properties on the GPU path
# ---------------------------------------------------------------------------

def test_linearity_of_forward():
    a = plane(64, 64, seed=1) // 2
    b = plane(64, 64, seed=2) // 2
    ya = host(R.forward(g(a), R.select(R.SEL_NONE), R.COEF_I32))
    yb = host(R.forward(g(b), R.select(R.SEL_NONE), R.COEF_I32))
    yab = host(R.forward(g(a + b), R.select(R.SEL_NONE), R.COEF_I32))
    assert np.array_equal(ya + yb, yab)


def test_full_retention_reconstructs_exactly():
    img = plane(64, 80, seed=5)
    sse, _, rec = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=64), 1, None, True)
    assert int(host(sse)[0]) == 0
    assert np.array_equal(host(rec), img.astype(np.float32))


def test_sweep_is_monotone_and_shift_invariant():
    img = plane(128, 128, seed=9)
    s, _, _ = R.compress_eval(g(img), R.select(R.SEL_ZIGZAG, r=1), 64)
    v = host(s)
    assert np.all(np.diff(v) <= 0) and v[-1] == 0
    shifted = (img.astype(np.int64) // 2 + 60).astype(np.uint8)
    half = (img.astype(np.int64) // 2).astype(np.uint8)
    a, _, _ = R.compress_eval(g(shifted), R.select(R.SEL_ZIGZAG, r=1), 45)
    b, _, _ = R.compress_eval(g(half), R.select(R.SEL_ZIGZAG, r=1), 45)
    assert np.array_equal(host(a), host(b))


def test_psnr_on_the_device_equals_the_host_call():
    # rdct_psnr_device forms the same decibels as rdct_psnr_planes (and the mean
    # over planes at every r), +inf for a zero sum, up to the last bits of the
    # two log10 implementations.
    rng = np.random.default_rng(21)
    n, rc = 37, 9
    widths = rng.integers(8, 600, n)
    heights = rng.integers(8, 600, n)
    sse = rng.integers(0, 2 ** 45, size=(n, rc)).astype(np.int64)
    sse[3, 4] = 0
    for mode in (R.SEL_ZIGZAG, R.SEL_QUANT):
        want, want_mean = R.rdct_psnr_planes(sse, rc, mode, widths, heights, mean=True)
        d_sse = torch.from_numpy(sse).to(DEV)
        pix = torch.from_numpy((widths * heights).astype(np.int64)).to(DEV)
        out = torch.empty(n * rc, dtype=torch.float64, device=DEV)
        mean = torch.empty(rc, dtype=torch.float64, device=DEV)
        R.rdct_psnr_device(d_sse, rc, mode, pix, out, mean)
        got = host(out).reshape(n, rc)
        assert np.isinf(got[3, 4]) and np.isinf(host(mean)[4])
        fin = np.isfinite(want)
        assert np.array_equal(fin, np.isfinite(got))
        assert np.max(np.abs(got[fin] - want[fin])) < 1e-11
        m = host(mean)
        ok = np.isfinite(want_mean)
        assert np.max(np.abs(m[ok] - want_mean[ok])) < 1e-11


@pytest.mark.parametrize("pattern", [R.STREAM_READ, R.STREAM_WRITE, R.STREAM_COPY, R.STREAM_R1W2,
                                     R.STREAM_R1W6])
@pytest.mark.parametrize("flags,wpc", [(0, 0), (3, 0), (2, 2), (7, 4)])
def test_stream_calibration_moves_what_it_says(pattern, flags, wpc):
    # The calibration kernel's stores: unit u's j-th KiB of output is the
    # (j mod RL)-th KiB of its input with every 32-bit word XORed with j (for
    # pure writes, the words (u, lane, 0, 0) XOR j); every unit is written once,
    # whatever the load / store kinds, the grid and the XCD order.
    rb, wb = R.rdct_stream_unit_bytes(pattern)
    units = 37
    src = torch.randint(0, 2 ** 31 - 1, (max(units * rb // 4, 4),), dtype=torch.int32, device=DEV)
    dst = torch.full((max(units * wb // 4, 256),), -1, dtype=torch.int32, device=DEV)
    R.rdct_stream(src if rb else None, dst, units, pattern, flags, wpc)
    torch.cuda.synchronize()
    if wb == 0:
        return   # reads only: the destination is written for one value of the data only
    rl, wl = rb // 1024, wb // 1024
    d = host(dst).view(np.uint32).reshape(units, wl, 64, 4)
    if rl:
        sv = host(src).view(np.uint32).reshape(units, rl, 64, 4)
        want = np.stack([sv[:, j % rl] ^ np.uint32(j) for j in range(wl)], axis=1)
    else:
        base = np.zeros((units, 64, 4), dtype=np.uint32)
        base[:, :, 0] = np.arange(units, dtype=np.uint32)[:, None]
        base[:, :, 1] = np.arange(64, dtype=np.uint32)[None, :]
        want = np.stack([base ^ np.uint32(j) for j in range(wl)], axis=1)
    assert np.array_equal(d, want)
