"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  Each pin is something other than the oracle
itself: a value printed in the paper (fixtures under tests/golden/, each citing
its passage), a closed form, an invariant, or brute force on tiny inputs.
"""
import itertools
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from conftest import read_golden

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------------------
# Constants (Section 2)
# ---------------------------------------------------------------------------

def test_c0_matches_printed_matrix():
    printed = np.array([[int(v) for v in row] for row in read_golden("c0_printed.txt")])
    assert printed.shape == (8, 8)
    assert np.array_equal(O.round_off_matrix(), printed)


def test_c0_rounding_has_no_ties():
    # Matlab rounding vs half-to-even give the same C0: no entry of 2C sits on .5.
    two_c = 2.0 * O.dct_matrix()
    frac = np.abs(two_c) - np.floor(np.abs(two_c))
    assert np.min(np.abs(frac - 0.5)) > 0.05
    assert np.array_equal(np.round(two_c).astype(np.int64), O.round_off_matrix())


def test_matlab_round_halves_away_from_zero():
    x = np.array([-2.5, -1.5, -0.5, 0.5, 1.5, 2.5, 2.49, -2.51])
    assert list(O.matlab_round(x)) == [-3, -2, -1, 1, 2, 3, 2, -3]


def test_dct_matrix_is_the_orthonormal_dct():
    c = O.dct_matrix()
    assert np.allclose(c @ c.T, np.eye(8), atol=1e-14)
    # Closed form of the first two rows.
    assert np.allclose(c[0], np.full(8, 1 / math.sqrt(8)))
    assert np.allclose(c[1], [0.5 * math.cos(math.pi * (2 * n + 1) / 16) for n in range(8)])


def test_gram_is_diagonal():
    g = O.gram()
    assert np.array_equal(g, np.diag([8, 6, 4, 6, 8, 6, 4, 6]))


def test_s_matches_printed_diagonal():
    rows = read_golden("s_printed.txt")
    printed = np.array([int(a) / (int(m) * math.sqrt(int(r))) for a, m, r in rows])
    s = O.orthogonalizer()
    assert np.allclose(np.diag(s), printed, atol=1e-15, rtol=0)
    assert np.allclose(s - np.diag(np.diag(s)), 0.0, atol=1e-15)


def test_c_orth_is_orthogonal():
    t = O.approx_dct()
    assert np.allclose(t @ t.T, np.eye(8), atol=1e-14)
    assert np.allclose(t.T @ t, np.eye(8), atol=1e-14)


def test_c0_alone_is_not_orthogonal():
    # Section 2 notes C0^-1 != C0^T.
    c0 = O.round_off_matrix().astype(float)
    assert not np.allclose(np.linalg.inv(c0), c0.T)


def test_frobenius_scale_matches_text():
    rows = dict((r[0], r[1]) for r in read_golden("scalars.txt"))
    assert round(O.frobenius_scale(), 4) == float(rows["frobenius_scale"])


def test_rows_0_and_4_coincide_with_dct():
    # Section 2: for m = 0, 4 the transfer functions equal the DCT's.
    t, c = O.approx_dct(), O.dct_matrix()
    assert np.allclose(t[0], c[0], atol=1e-15)
    assert np.allclose(t[4], c[4], atol=1e-15)
    for m in range(8):
        if m not in (0, 4):
            assert not np.allclose(t[m], c[m], atol=1e-3)


def _table2():
    rows = read_golden("table2_error_energy.txt")
    return {r[0]: [float(v) for v in r[1:]] for r in rows}


def test_table2_proposed_column():
    tab = _table2()
    t = O.approx_dct()
    total = 0.0
    for m in (1, 2, 3, 5, 6, 7):
        e = O.error_energy(m, t)
        total += e
        assert round(e, 2) == tab[str(m)][3], m
    for m in (0, 4):
        assert O.error_energy(m, t) < 1e-20
    assert round(total, 2) == tab["total"][3]


def test_table2_sdct_column():
    tab = _table2()
    t = O.sdct_matrix()
    total = sum(O.error_energy(m, t) for m in range(8))
    for m in (1, 2, 3, 5, 6, 7):
        assert round(O.error_energy(m, t), 2) == tab[str(m)][2], m
    assert round(total, 2) == tab["total"][2]


def test_error_energy_closed_form():
    # For an FIR difference d, int_0^pi |sum d_n e^{-jnw}|^2 dw = pi ||d||^2.
    c = O.dct_matrix()
    for t in (O.approx_dct(), O.sdct_matrix()):
        for m in range(8):
            assert abs(O.error_energy(m, t) - math.pi * np.sum((c[m] - t[m]) ** 2)) < 1e-9


# ---------------------------------------------------------------------------
# Fast algorithm (Fig. 1, Table 1)
# ---------------------------------------------------------------------------

def test_fast_algorithm_operation_count_matches_table1():
    rows = {r[0]: [int(v) for v in r[1:]] for r in read_golden("table1_complexity.txt")}
    ops = O.OpCounter()
    O.fast_c0_1d(list(range(8)), ops)
    assert (ops.add, ops.mul, ops.shift) == tuple(rows["proposed"][:3])
    ops_t = O.OpCounter()
    O.fast_c0t_1d(list(range(8)), ops_t)
    assert (ops_t.add, ops_t.mul, ops_t.shift) == (22, 0, 0)


def test_fast_algorithm_equals_c0_on_all_ternary_vectors():
    c0 = O.round_off_matrix()
    x = np.array(list(itertools.product((-1, 0, 1), repeat=8)), dtype=np.int64).T  # 8 x 6561
    fast = np.array(O.fast_c0_1d(x))
    assert np.array_equal(fast, c0 @ x)
    fast_t = np.array(O.fast_c0t_1d(x))
    assert np.array_equal(fast_t, c0.T @ x)


def test_fast_algorithm_on_basis_and_random_bytes():
    c0 = O.round_off_matrix()
    for j in range(8):
        e = [0] * 8
        e[j] = 1
        assert O.fast_c0_1d(e) == list(c0[:, j])
    x = RNG.integers(0, 256, size=(8, 1000))
    assert np.array_equal(np.array(O.fast_c0_1d(x)), c0 @ x)


# ---------------------------------------------------------------------------
# 2-D forward transform (Section 3)
# ---------------------------------------------------------------------------

def _brute_forward(a):
    c0 = O.round_off_matrix().tolist()
    y = [[0] * 8 for _ in range(8)]
    for k in range(8):
        for l in range(8):
            s = 0
            for i in range(8):
                for j in range(8):
                    s += c0[k][i] * int(a[i][j]) * c0[l][j]
            y[k][l] = s
    return np.array(y)


def test_forward_matches_brute_force():
    for _ in range(5):
        a = RNG.integers(0, 256, size=(8, 8))
        assert np.array_equal(O.forward_blocks(a), _brute_forward(a))


def test_forward_orientation():
    # A[i, j] = j varies horizontally only: energy must sit in row k = 0 of Y
    # (k = vertical frequency).  A transposed operand would put it in column 0.
    a = np.tile(np.arange(8), (8, 1))
    y = O.forward_blocks(a)
    assert np.all(y[1:, :] == 0) and np.any(y[0, 1:] != 0)
    y2 = O.forward_blocks(a.T)
    assert np.all(y2[:, 1:] == 0) and np.any(y2[1:, 0] != 0)


def test_forward_constant_blocks_and_level_shift():
    a = np.full((8, 8), 255)
    y = O.forward_blocks(a)
    assert y[0, 0] == 16320 and np.count_nonzero(y) == 1
    ys = O.forward_blocks(a, level_shift=128)
    assert ys[0, 0] == 64 * 127 and np.count_nonzero(ys) == 1
    # Rows 1-7 of C0 sum to zero, so a shift only moves the DC term.
    b = RNG.integers(0, 256, size=(8, 8))
    d = O.forward_blocks(b) - O.forward_blocks(b, level_shift=128)
    assert d[0, 0] == 8192 and np.count_nonzero(d) == 1


def test_forward_range_bound():
    # |Y_kl| <= 255 * (number of (i, j) with C0[k,i] C0[l,j] > 0), reached by the
    # block that is 255 exactly there and 0 elsewhere.
    c0 = O.round_off_matrix()
    for k in range(8):
        for l in range(8):
            pos = (np.outer(c0[k], c0[l]) > 0).astype(np.int64)
            y = O.forward_blocks(255 * pos)
            assert y[k, l] == 255 * pos.sum()
            assert y[k, l] <= 16320


# ---------------------------------------------------------------------------
# Selection (Section 3 zig-zag; quantisation reading)
# ---------------------------------------------------------------------------

def test_zigzag_is_the_standard_sequence():
    zz = O.zigzag_order()
    assert len(set(zz)) == 64
    assert zz[:10] == [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2), (0, 3), (1, 2), (2, 1), (3, 0)]
    assert zz[-3:] == [(7, 6), (6, 7), (7, 7)] or zz[-3:] == [(6, 7), (7, 6), (7, 7)]
    assert zz[-1] == (7, 7)
    for (k0, l0), (k1, l1) in zip(zz, zz[1:]):
        assert max(abs(k1 - k0), abs(l1 - l0)) == 1       # neighbouring positions
        assert k1 + l1 in (k0 + l0, k0 + l0 + 1)           # anti-diagonals in order


def test_zigzag_masks():
    assert O.retention_mask(64).sum() == 64
    assert O.retention_mask(1).sum() == 1 and O.retention_mask(1)[0, 0] == 1
    for r in (1, 3, 6, 10, 15, 21, 28, 36):   # whole anti-diagonals kept
        m = O.retention_mask(r)
        assert np.array_equal(m, m.T)
    for r in (2, 4, 5, 7, 9, 45):
        m = O.retention_mask(r)
        assert not np.array_equal(m, m.T)
    assert O.retention_mask(2)[0, 1] == 1 and O.retention_mask(2)[1, 0] == 0


def test_quant_table_golden_and_scaling():
    q50 = np.array([[int(v) for v in r] for r in read_golden("jpeg_luma_q50.txt")])
    assert np.array_equal(O.quant_table(50), q50)
    assert np.all(O.quant_table(100) == 1)
    assert np.all(O.quant_table(1) == 255)   # f = 5000 saturates every entry
    prev = None
    for q in range(1, 101):
        t = O.quant_table(q)
        assert t.min() >= 1 and t.max() <= 255
        if prev is not None:
            assert np.all(t <= prev)
        prev = t


def _libjpeg_luma_table(quality):
    """The luminance table libjpeg writes at `quality`: a 16 x 16 grey image saved
    through Pillow at that quality and read back (natural order, k = row)."""
    import io
    from PIL import Image
    buf = io.BytesIO()
    Image.fromarray(np.zeros((16, 16), dtype=np.uint8)).save(buf, "JPEG", quality=quality)
    buf.seek(0)
    return np.array(Image.open(buf).quantization[0], dtype=np.int64).reshape(8, 8)


def test_quant_table_matches_libjpeg_at_every_quality():
    # The IJG quality rule as libjpeg implements it (an independent program):
    # its rounding term, the integer 5000 / q and the clamps all show somewhere
    # in 1..100, where quality 50 alone would not reveal them.
    for q in range(1, 101):
        assert np.array_equal(O.quant_table(q), _libjpeg_luma_table(q)), f"quality {q}"


def _exact_round_half_away(y, q, gkk, gll):
    # round(y / (q sqrt(gkk gll))) with 60-digit decimal arithmetic.
    getcontext().prec = 60
    x = Decimal(y) / (Decimal(q) * (Decimal(gkk * gll)).sqrt())
    n = (abs(x) + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR")
    return int(n) if y >= 0 else -int(n)


def test_quantize_matches_exact_decimal_rounding():
    g = np.diag(O.gram())
    positions = [(0, 0), (0, 4), (1, 1), (0, 1), (0, 2), (1, 2), (2, 2), (3, 5), (6, 7)]
    for (k, l) in positions:
        for qv in (1, 3, 7, 16, 61):
            ys = np.arange(-1200, 1201)
            qtab = np.full((8, 8), qv)
            ymat = np.zeros((ys.size, 8, 8), dtype=np.int64)
            ymat[:, k, l] = ys
            got = O.quantize(ymat, qtab)[:, k, l]
            want = [_exact_round_half_away(int(y), qv, int(g[k]), int(g[l])) for y in ys]
            assert list(got) == want, (k, l, qv)


def test_quantize_exact_ties_round_away_from_zero():
    # Position (1, 1): s_1 s_1 = 1/6, so z/Q = Y / (6 Q); Y = 3 Q (2n + 1) is a tie.
    qtab = np.full((8, 8), 5)
    for n in range(0, 40):
        for sgn in (1, -1):
            y = np.zeros((8, 8), dtype=np.int64)
            y[1, 1] = sgn * 3 * 5 * (2 * n + 1)
            assert O.quantize(y, qtab)[1, 1] == sgn * (n + 1)
            assert Fraction(int(y[1, 1]), 30) == sgn * Fraction(2 * n + 1, 2)


# ---------------------------------------------------------------------------
# Inverse and metrics
# ---------------------------------------------------------------------------

def test_d_prime_identity_exact():
    # C0^T diag(d'/24) C0 = I exactly (S^2 = diag(d') / 24).
    c0 = O.round_off_matrix().tolist()
    d = O.d_prime().tolist()
    assert d == [3, 4, 6, 4, 3, 4, 6, 4]
    for i in range(8):
        for j in range(8):
            s = sum(Fraction(c0[k][i] * d[k] * c0[k][j], 24) for k in range(8))
            assert s == (1 if i == j else 0)


def test_perfect_reconstruction_with_all_coefficients():
    a = RNG.integers(0, 256, size=(20, 8, 8))
    y = O.forward_blocks(a)
    assert np.array_equal(O.retention_numerator(y, 64), 576 * a)
    assert np.allclose(O.inverse_orth(O.scale_coeffs(y)), a, atol=1e-10)


def test_retention_numerator_equals_orthogonal_inverse():
    a = RNG.integers(0, 256, size=(10, 8, 8))
    y = O.forward_blocks(a)
    for r in (1, 5, 10, 33, 45):
        via_int = O.retention_numerator(y, r) / 576.0
        via_def = O.inverse_orth(O.scale_coeffs(y) * O.retention_mask(r))
        assert np.allclose(via_int, via_def, atol=1e-10)


def test_parseval_in_integers_for_every_r():
    a = RNG.integers(0, 256, size=(12, 8, 8))
    y = O.forward_blocks(a)
    dp = O.d_prime()
    w = np.outer(dp, dp)
    for r in range(0, 65):
        e = 576 * a - O.retention_numerator(y, r)
        lhs = np.sum(e * e, axis=(1, 2))
        rhs = 576 * np.sum(w * y * y * (1 - O.retention_mask(r)), axis=(1, 2))
        assert np.array_equal(lhs, rhs), r


def test_sse_monotone_and_constant_plane():
    img = RNG.integers(0, 256, size=(24, 40)).astype(np.uint8)
    res = O.retention_eval(img, range(1, 65))
    vals = [res["sse_num"][r] for r in range(1, 65)]
    assert all(b <= a for a, b in zip(vals, vals[1:]))
    assert vals[-1] == 0 and res["psnr"][64] == float("inf")
    const = np.full((16, 24), 77, dtype=np.uint8)
    rc = O.retention_eval(const, range(1, 46))
    assert all(rc["sse_num"][r] == 0 for r in range(1, 46))


def test_psnr_values():
    assert O.psnr_from_mse(0.0) == float("inf")
    assert abs(O.psnr_from_mse(255.0 ** 2)) < 1e-12
    assert abs(O.psnr_from_mse(255.0 ** 2 / 100.0) - 20.0) < 1e-12
    assert O.average_psnr([10.0, 20.0, 33.0]) == 21.0


def test_quant_path_error_equals_coefficient_error():
    # Orthogonality: ||A - A'||^2 = ||Z - Z'||^2 for the quantisation path.
    img = RNG.integers(0, 256, size=(32, 48)).astype(np.uint8)
    qt = O.quant_table(37)
    res = O.quant_eval(img, qt)
    z = O.scale_coeffs(res["Y"])
    zq = O.dequantize(res["q"], qt)
    assert abs(res["sse"] - np.sum((z - zq) ** 2)) < 1e-8 * max(1.0, res["sse"])


def test_quant_with_unit_table_at_quality_100_is_near_lossless():
    img = RNG.integers(0, 256, size=(16, 16)).astype(np.uint8)
    res = O.quant_eval(img, O.quant_table(100))
    # Rounding each C_orth coefficient to an integer: per-pixel MSE <= 1/4.
    assert res["mse"] <= 0.25


# ---------------------------------------------------------------------------
# Tiling and whole-plane pipelines against pure-python loops
# ---------------------------------------------------------------------------

def test_tiling_edge_replication():
    img = np.arange(11 * 13).reshape(11, 13).astype(np.uint8)
    b = O.tile(img)
    assert b.shape == (2, 2, 8, 8)
    assert b[1, 1, 7, 7] == img[10, 12]
    assert b[1, 0, 5, 3] == img[10, 3]   # row 13 -> replicated row 10
    assert np.array_equal(O.untile(b, 11, 13), img)
    m = O.valid_mask(11, 13)
    assert m.sum() == 11 * 13


def _loop_retention(img, r):
    """Pure-python reconstruction with C_orth^T (M_r . Z) C_orth in float64."""
    h, w = img.shape
    t = O.approx_dct().tolist()
    rank = O.zigzag_rank().tolist()
    rec = np.zeros((h, w))
    for by in range(0, h, 8):
        for bx in range(0, w, 8):
            a = [[int(img[min(by + i, h - 1)][min(bx + j, w - 1)]) for j in range(8)] for i in range(8)]
            z = [[sum(t[k][i] * a[i][j] * t[l][j] for i in range(8) for j in range(8))
                  if rank[k][l] < r else 0.0 for l in range(8)] for k in range(8)]
            for i in range(8):
                for j in range(8):
                    if by + i < h and bx + j < w:
                        rec[by + i, bx + j] = sum(t[k][i] * z[k][l] * t[l][j]
                                                  for k in range(8) for l in range(8))
    return rec


def test_retention_pipeline_matches_loops():
    img = RNG.integers(0, 256, size=(12, 20)).astype(np.uint8)
    for r in (1, 5, 10):
        res = O.retention_eval(img, [r], recon_r=r)
        ref = _loop_retention(img, r)
        assert np.allclose(res["recon"], ref, atol=1e-9)
        sse = float(np.sum((img.astype(float) - ref) ** 2))
        assert abs(res["sse"][r] - sse) < 1e-6 * max(1.0, sse)
        assert abs(res["psnr"][r] - 10 * math.log10(255 ** 2 * img.size / sse)) < 1e-9


def test_quant_pipeline_matches_loops():
    img = RNG.integers(0, 256, size=(8, 16)).astype(np.uint8)
    qt = O.quant_table(50)
    res = O.quant_eval(img, qt)
    t = O.approx_dct().tolist()
    g = np.diag(O.gram()).tolist()
    for bx in range(2):
        a = [[int(img[i][8 * bx + j]) - 128 for j in range(8)] for i in range(8)]
        for k in range(8):
            for l in range(8):
                z = sum(t[k][i] * a[i][j] * t[l][j] for i in range(8) for j in range(8))
                y = int(res["Y"][0, bx, k, l])
                assert abs(z - y / math.sqrt(g[k] * g[l])) < 1e-9
                assert res["q"][0, bx, k, l] == _exact_round_half_away(y, int(qt[k, l]), g[k], g[l])


def test_quant_reconstruction_matches_loops():
    # The dequantised reconstruction A' = C_orth^T (q . Q) C_orth + 128 and its
    # SSE, by pure-python loops over k, l, i, j, at tables that are not symmetric
    # (a transposed table or a transposed inverse changes the result), plus the
    # quantiser's bound |Z - q Q| <= Q / 2 per coefficient.
    img = RNG.integers(0, 256, size=(16, 24)).astype(np.uint8)
    t = O.approx_dct().tolist()
    for quality in (50, 23, 81):
        qt = O.quant_table(quality)
        assert not np.array_equal(qt, qt.T)
        res = O.quant_eval(img, qt)
        sse = 0.0
        for by in range(2):
            for bx in range(3):
                a = [[int(img[8 * by + i][8 * bx + j]) for j in range(8)] for i in range(8)]
                q = res["q"][by, bx].tolist()
                for k in range(8):
                    for l in range(8):
                        z = sum(t[k][i] * (a[i][j] - 128) * t[l][j]
                                for i in range(8) for j in range(8))
                        assert abs(z - q[k][l] * int(qt[k, l])) <= qt[k, l] / 2 + 1e-9
                for i in range(8):
                    for j in range(8):
                        rec = 128.0 + sum(t[k][i] * (q[k][l] * int(qt[k, l])) * t[l][j]
                                          for k in range(8) for l in range(8))
                        assert abs(res["recon"][8 * by + i, 8 * bx + j] - rec) < 1e-9
                        sse += (a[i][j] - rec) ** 2
        assert abs(res["sse"] - sse) < 1e-9 * max(1.0, sse)
