"""Spectral error of approximate transforms (Section 2, Table 2).

Test infrastructure only (see the package docstring).  Used to pin the oracle's
constants against the printed error energies: each row t_m of a transform T is
read as an FIR filter with transfer function H_m(w; T) = sum_n t_{m,n} e^{-j n w};
D_m(w; T) = |H_m(w; C) - H_m(w; T)|^2 and eps_m(T) is its integral over [0, pi],
evaluated numerically as in the paper.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate

from . import rdct


def transfer(row: np.ndarray, w: np.ndarray) -> np.ndarray:
    """H_m(w) = sum_n t_{m,n} exp(-j n w) for one row t_m."""
    n = np.arange(len(row))
    return np.exp(-1j * np.outer(np.atleast_1d(w), n)) @ np.asarray(row, dtype=np.float64)


def sq_mag_error(m: int, t: np.ndarray, w) -> np.ndarray:
    """D_m(w; T) = |H_m(w; C) - H_m(w; T)|^2."""
    c = rdct.dct_matrix()
    return np.abs(transfer(c[m], w) - transfer(t[m], w)) ** 2


def error_energy(m: int, t: np.ndarray) -> float:
    """eps_m(T) = integral_0^pi D_m(w; T) dw, by adaptive quadrature."""
    val, _ = integrate.quad(lambda w: float(sq_mag_error(m, t, w)[0]), 0.0, np.pi,
                            limit=200, epsabs=1e-12, epsrel=1e-12)
    return float(val)


def sdct_matrix() -> np.ndarray:
    """The signed DCT comparator of Section 2: sign(C) / sqrt(8)."""
    return np.sign(rdct.dct_matrix()) / np.sqrt(8.0)


__all__ = ["transfer", "sq_mag_error", "error_energy", "sdct_matrix"]
