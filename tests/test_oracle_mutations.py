"""Planted mistakes in the oracle (CPU only): each must make a pin fail.

A pin set that a plausible slip (a transposed operand, a wrong sign, a dropped
term, a swapped traversal, a different tie rule) survives would not be a pin.
"""
import numpy as np
import pytest

import oracle as O
import oracle.rdct as R
import test_oracle_pins as P


def _fails(pin):
    with pytest.raises(AssertionError):
        pin()


def test_transposed_operand_in_forward_is_caught(monkeypatch):
    def bad(blocks, level_shift=0):
        c0 = R.round_off_matrix()
        a = np.asarray(blocks).astype(np.int64) - level_shift
        return np.matmul(np.matmul(c0, np.swapaxes(a, -1, -2)), c0.T)
    monkeypatch.setattr(R, "forward_blocks", bad)
    monkeypatch.setattr(O, "forward_blocks", bad)
    _fails(P.test_forward_orientation)


def test_sign_slip_in_fast_algorithm_is_caught(monkeypatch):
    good = R.fast_c0_1d

    def bad(x, ops=None):
        out = good(x, ops)
        out[6] = -out[6]
        return out
    monkeypatch.setattr(O, "fast_c0_1d", bad)
    _fails(P.test_fast_algorithm_equals_c0_on_all_ternary_vectors)


def test_dropped_term_in_fast_algorithm_is_caught(monkeypatch):
    good = R.fast_c0_1d

    def bad(x, ops=None):
        out = good(x, ops)
        out[3] = out[3] + x[3]          # b3 dropped from X3
        return out
    monkeypatch.setattr(O, "fast_c0_1d", bad)
    _fails(P.test_fast_algorithm_equals_c0_on_all_ternary_vectors)


def test_swapped_zigzag_direction_is_caught(monkeypatch):
    good = R.zigzag_order

    def bad():
        return [(l, k) for (k, l) in good()]
    monkeypatch.setattr(O, "zigzag_order", bad)
    _fails(P.test_zigzag_is_the_standard_sequence)


def test_half_even_quantiser_is_caught(monkeypatch):
    def bad(y, qtab):
        g = np.diag(R.gram())
        z = np.asarray(y, dtype=np.float64) / (qtab * np.sqrt(np.outer(g, g)))
        return np.round(z).astype(np.int64)
    monkeypatch.setattr(O, "quantize", bad)
    _fails(P.test_quantize_exact_ties_round_away_from_zero)


def test_wrong_orthogonaliser_is_caught(monkeypatch):
    def bad(c0=None):
        s = np.diag(1.0 / np.sqrt(np.diag(R.gram()).astype(float)))
        s[2, 2] = 1 / np.sqrt(6.0)
        return s
    monkeypatch.setattr(O, "orthogonalizer", bad)
    _fails(P.test_s_matches_printed_diagonal)


def test_wrong_inverse_weights_are_caught(monkeypatch):
    monkeypatch.setattr(R, "d_prime", lambda: np.array([3, 4, 6, 4, 3, 4, 4, 6]))
    _fails(P.test_perfect_reconstruction_with_all_coefficients)


def test_reconstruction_without_transpose_is_caught(monkeypatch):
    def bad(z):
        t = R.approx_dct()
        return np.matmul(np.matmul(t, np.asarray(z, dtype=np.float64)), t.T)
    monkeypatch.setattr(O, "inverse_orth", bad)
    _fails(P.test_perfect_reconstruction_with_all_coefficients)


# --- comparison transforms and UQI ---------------------------------------------------

import oracle.quality as Q  # noqa: E402
import test_oracle_quality_pins as QP  # noqa: E402


def test_uqi_with_mismatched_normalisation_is_caught(monkeypatch):
    good = Q.uqi_map

    def bad(x, y, win=8):
        # variances over n, covariance over n - 1
        return good(x, y, win) * (win * win) / (win * win - 1)
    monkeypatch.setattr(O, "uqi_map", bad)
    _fails(QP.test_uqi_identical_is_one_and_window_count)


def test_uqi_mean_factor_typo_is_caught(monkeypatch):
    def bad(x, y, win=8):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        xw = np.lib.stride_tricks.sliding_window_view(x, (win, win))
        yw = np.lib.stride_tricks.sliding_window_view(y, (win, win))
        mx, my = xw.mean(axis=(2, 3)), yw.mean(axis=(2, 3))
        dx, dy = xw - mx[..., None, None], yw - my[..., None, None]
        vx, vy = (dx * dx).mean(axis=(2, 3)), (dy * dy).mean(axis=(2, 3))
        cxy = (dx * dy).mean(axis=(2, 3))
        return (2 * cxy / (vx + vy)) * (2 * mx * my / (mx * mx + my * mx))
    monkeypatch.setattr(O, "uqi_map", bad)
    _fails(QP.test_uqi_shifted_copy_closed_form)


def test_missing_transpose_in_inverse_is_caught(monkeypatch):
    def bad(img, name, r):
        img = np.asarray(img)
        h, w = img.shape
        t, ti = Q.transform(name)
        a = O.tile(img).astype(np.float64)
        y = np.matmul(np.matmul(t, a), t.T) * O.retention_mask(r)
        return O.untile(np.matmul(np.matmul(ti, y), ti), h, w)
    monkeypatch.setattr(O, "retention_recon", bad)
    _fails(lambda: QP.test_all_coefficients_reconstruct_exactly("sdct"))


def test_transposed_retention_mask_is_caught(monkeypatch):
    def bad(img, name, r):
        img = np.asarray(img)
        h, w = img.shape
        t, ti = Q.transform(name)
        a = O.tile(img).astype(np.float64)
        y = np.matmul(np.matmul(t, a), t.T) * O.retention_mask(r).T
        return O.untile(np.matmul(np.matmul(ti, y), ti.T), h, w)
    monkeypatch.setattr(Q, "retention_recon", bad)
    _fails(QP.test_dct_sse_is_parseval_of_dropped_coefficients)


# --- codec output ------------------------------------------------------------

import oracle.codec as CD  # noqa: E402
import test_oracle_codec_pins as CP  # noqa: E402


def test_run_off_by_one_is_caught(monkeypatch):
    def bad(values):
        pairs, run = [], 0
        for v in values:
            run += 1
            if int(v) != 0:
                pairs.append((run, int(v)))
                run = 0
        return pairs
    monkeypatch.setattr(O, "rle_encode", bad)
    _fails(CP.test_rle_hand_examples)


def test_half_even_pixel_rounding_is_caught(monkeypatch):
    def bad(r_num):
        return np.clip(np.rint(np.asarray(r_num) / 576.0), 0, 255).astype(np.uint8)
    monkeypatch.setattr(O, "u8_from_numerator", bad)
    _fails(CP.test_u8_rounding_is_half_away_and_clamped)


def test_transposed_table_in_dequantize_is_caught(monkeypatch):
    def bad(q, qtab):
        return np.asarray(q, dtype=np.float64) * np.asarray(qtab, dtype=np.float64).T
    monkeypatch.setattr(R, "dequantize", bad)
    monkeypatch.setattr(O, "dequantize", bad)
    _fails(P.test_quant_reconstruction_matches_loops)


def test_dropped_rounding_term_in_quant_table_is_caught(monkeypatch):
    def bad(quality):
        f = 5000 // quality if quality < 50 else 200 - 2 * quality
        return np.clip((R.JPEG_LUMA_Q50 * f) // 100, 1, 255).astype(np.int64)
    monkeypatch.setattr(R, "quant_table", bad)
    monkeypatch.setattr(O, "quant_table", bad)
    _fails(P.test_quant_table_matches_libjpeg_at_every_quality)


def test_float_quality_factor_in_quant_table_is_caught(monkeypatch):
    def bad(quality):
        f = 5000 / quality if quality < 50 else 200 - 2 * quality
        return np.clip(np.floor((R.JPEG_LUMA_Q50 * f + 50) / 100), 1, 255).astype(np.int64)
    monkeypatch.setattr(R, "quant_table", bad)
    monkeypatch.setattr(O, "quant_table", bad)
    _fails(P.test_quant_table_matches_libjpeg_at_every_quality)
