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
