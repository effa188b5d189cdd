"""Block-level oracle: constants, forward transform, selection, inverse, metrics.

Test infrastructure only (see the package docstring).

Notation follows the paper: C is the 8-point DCT matrix, C0 = [2 C] the round-off
matrix, S the diagonal orthogonaliser and C_orth = S C0 the proposed orthogonal
approximation (Section 2).  An 8x8 block A maps to Y = C0 A C0^T and to the
C_orth coefficients Z = S Y S (Section 3, the 2-D transform T A T^T with S merged
into the following quantisation step, Section 2).  Index convention: A[i, j] has
i = row, j = column; Y[k, l] has k = vertical and l = horizontal frequency.

Readings where the paper is silent (each is listed in the design notes):
  * C is the orthonormal type-II DCT (it reproduces the printed C0 and S).
  * Zig-zag order is the JPEG one: anti-diagonals t = k + l in increasing order,
    odd t traversed with k increasing, even t with k decreasing; its first step
    goes to (k, l) = (0, 1).
  * Quantisation divides Z by a quant table Q and rounds half away from zero,
    decided exactly; the table is the JPEG luminance table scaled by the IJG
    quality rule.  The quantisation path subtracts 128 from every pixel first.
  * Reconstruction is real-valued (no rounding or clipping before the metric);
    PSNR uses peak 255, MSE over the image's own pixels, +inf when MSE = 0.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import sqrtm

N = 8

# ---------------------------------------------------------------------------
# Constants (Section 2)
# ---------------------------------------------------------------------------


def dct_matrix(n: int = N) -> np.ndarray:
    """The standard orthonormal DCT-II matrix C (Sections 1-2):
    C[k, m] = alpha_k cos(pi (2m + 1) k / (2n)), alpha_0 = sqrt(1/n), else sqrt(2/n)."""
    k = np.arange(n, dtype=np.float64)[:, None]
    m = np.arange(n, dtype=np.float64)[None, :]
    alpha = np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
    return alpha * np.cos(np.pi * (2.0 * m + 1.0) * k / (2.0 * n))


def matlab_round(x):
    """The round-off operator [.] of Section 2 (Matlab's round): nearest integer,
    halves away from zero."""
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def round_off_matrix() -> np.ndarray:
    """C0 = [2 C] (Section 2, displayed matrix).  Entries are 0 or +-1."""
    return matlab_round(2.0 * dct_matrix()).astype(np.int64)


def gram(c0: np.ndarray | None = None) -> np.ndarray:
    """C0 C0^T as exact integers (Section 2, polar-decomposition step)."""
    c0 = round_off_matrix() if c0 is None else c0
    return c0 @ c0.T


def orthogonalizer(c0: np.ndarray | None = None) -> np.ndarray:
    """S = sqrt((C0 C0^T)^(-1)) with the principal matrix square root (Section 2)."""
    g = gram(c0).astype(np.float64)
    s = sqrtm(np.linalg.inv(g))
    return np.real_if_close(s).astype(np.float64)


def s_diag() -> np.ndarray:
    """Diagonal of S, i.e. (C0 C0^T)^(-1/2) for the diagonal Gram matrix."""
    return np.diag(orthogonalizer()).copy()


def approx_dct() -> np.ndarray:
    """C_orth = S C0, the proposed orthogonal approximation (Section 2)."""
    return orthogonalizer() @ round_off_matrix().astype(np.float64)


def frobenius_scale(c0: np.ndarray | None = None) -> float:
    """The scalar alpha minimising ||C - alpha C0||_F (Section 2 quotes 0.3922)."""
    c0 = round_off_matrix() if c0 is None else c0
    c = dct_matrix()
    c0 = c0.astype(np.float64)
    return float(np.sum(c * c0) / np.sum(c0 * c0))


# ---------------------------------------------------------------------------
# Fast algorithm for C0 (Section 2, Fig. 1 and Table 1: 22 additions)
# ---------------------------------------------------------------------------


class OpCounter:
    """Counts additions, multiplications and shifts used by a flow graph."""

    def __init__(self):
        self.add = 0
        self.mul = 0
        self.shift = 0

    def a(self, x, y):
        self.add += 1
        return x + y

    def s(self, x, y):
        self.add += 1
        return x - y


def fast_c0_1d(x, ops: OpCounter | None = None):
    """C0 x by an addition-only flow graph (our reading of Fig. 1, whose drawing is
    not in the text): the first stage forms sums a_i = x_i + x_{7-i} and
    differences b_i = x_i - x_{7-i}; the even outputs use the sums, the odd
    outputs use the differences.  Works on python ints or numpy arrays (the first
    axis indexes the 8 inputs).  Table 1 gives 22 additions, no multiplication and
    no shift; `ops` counts them."""
    o = ops if ops is not None else OpCounter()
    a = [o.a(x[i], x[7 - i]) for i in range(4)]
    b = [o.s(x[i], x[7 - i]) for i in range(4)]
    p03 = o.a(a[0], a[3])
    p12 = o.a(a[1], a[2])
    X0 = o.a(p03, p12)
    X4 = o.s(p03, p12)
    X2 = o.s(a[0], a[3])
    X6 = o.s(a[2], a[1])
    X1 = o.a(o.a(b[0], b[1]), b[2])
    X3 = o.s(o.s(b[0], b[2]), b[3])
    X5 = o.a(o.s(b[0], b[1]), b[3])
    X7 = o.s(o.s(b[2], b[1]), b[3])
    return [X0, X1, X2, X3, X4, X5, X6, X7]


def fast_c0t_1d(X, ops: OpCounter | None = None):
    """C0^T X by the transposed flow graph (22 additions); the inverse transform
    runs through the transpose because C_orth is orthogonal (Section 2)."""
    o = ops if ops is not None else OpCounter()
    p = o.a(X[0], X[4])
    m = o.s(X[0], X[4])
    a0 = o.a(p, X[2])
    a3 = o.s(p, X[2])
    a1 = o.s(m, X[6])
    a2 = o.a(m, X[6])
    b0 = o.a(o.a(X[1], X[3]), X[5])
    b1 = o.s(o.s(X[1], X[5]), X[7])
    b2 = o.a(o.s(X[1], X[3]), X[7])
    b3 = o.s(o.s(X[5], X[3]), X[7])
    a = [a0, a1, a2, a3]
    b = [b0, b1, b2, b3]
    out = [None] * 8
    for i in range(4):
        out[i] = o.a(a[i], b[i])
        out[7 - i] = o.s(a[i], b[i])
    return out


# ---------------------------------------------------------------------------
# 2-D block transform (Section 3: T A T^T on 8x8 sub-blocks)
# ---------------------------------------------------------------------------


def forward_blocks(blocks: np.ndarray, level_shift: int = 0) -> np.ndarray:
    """Y = C0 (A - shift) C0^T for a stack of 8x8 blocks (..., 8, 8), exact int64
    (Section 3, with T = C0; S is folded into the following step, Section 2)."""
    c0 = round_off_matrix()
    a = np.asarray(blocks).astype(np.int64) - int(level_shift)
    return np.matmul(np.matmul(c0, a), c0.T)


def scale_coeffs(y: np.ndarray) -> np.ndarray:
    """Z = S Y S: the C_orth coefficients z_kl = s_k s_l Y_kl in float64 (Section 2)."""
    s = s_diag()
    return np.asarray(y, dtype=np.float64) * np.outer(s, s)


def zigzag_order() -> list[tuple[int, int]]:
    """The standard zig-zag sequence of the 64 positions (Section 3; JPEG reading):
    anti-diagonals t = k + l in increasing order, odd t with k increasing and even
    t with k decreasing."""
    order = []
    for t in range(2 * N - 1):
        ks = [k for k in range(N) if 0 <= t - k < N]
        ks = ks if t % 2 == 1 else ks[::-1]
        order.extend((k, t - k) for k in ks)
    return order


def zigzag_rank() -> np.ndarray:
    """rank[k, l] = position of (k, l) in the zig-zag sequence."""
    rank = np.empty((N, N), dtype=np.int64)
    for i, (k, l) in enumerate(zigzag_order()):
        rank[k, l] = i
    return rank


def retention_mask(r: int) -> np.ndarray:
    """M_r[k, l] = 1 for the r initial zig-zag positions, 0 for the rest
    (Section 3: only the r initial coefficients are retained, 1 <= r <= 45 there)."""
    if not 0 <= r <= N * N:
        raise ValueError("r out of range")
    return (zigzag_rank() < r).astype(np.int64)


# --- quantisation (S folded into the quantisation, Section 2) ----------------

# JPEG luminance quant table for quality 50 (ITU-T T.81 Annex K, Table K.1),
# natural order, row index = vertical frequency k.
JPEG_LUMA_Q50 = np.array([
    [16, 11, 10, 16, 24, 40, 51, 61],
    [12, 12, 14, 19, 26, 58, 60, 55],
    [14, 13, 16, 24, 40, 57, 69, 56],
    [14, 17, 22, 29, 51, 87, 80, 62],
    [18, 22, 37, 56, 68, 109, 103, 77],
    [24, 35, 55, 64, 81, 104, 113, 92],
    [49, 64, 78, 87, 103, 121, 120, 101],
    [72, 92, 95, 98, 112, 100, 103, 99],
], dtype=np.int64)


def quant_table(quality: int) -> np.ndarray:
    """IJG quality scaling of the luminance table: f = 5000 // q for q < 50, else
    200 - 2 q; Q = clamp((Q50 f + 50) // 100, 1, 255)."""
    if not 1 <= quality <= 100:
        raise ValueError("quality must be in 1..100")
    f = 5000 // quality if quality < 50 else 200 - 2 * quality
    return np.clip((JPEG_LUMA_Q50 * f + 50) // 100, 1, 255).astype(np.int64)


def quantize(y: np.ndarray, qtab: np.ndarray) -> np.ndarray:
    """q_kl = round(z_kl / Q_kl) with z = S Y S, halves away from zero, decided
    exactly.  Since z_kl / Q_kl = Y_kl / (Q_kl sqrt(G_kk G_ll)), |q| is the largest
    n >= 0 with n = 0 or 4 Y^2 >= (2n - 1)^2 Q^2 G_kk G_ll (all integers).  A
    float64 estimate picks n, integer tests correct it."""
    y = np.asarray(y, dtype=np.int64)
    g = np.diag(gram())
    gg = np.outer(g, g)                       # G_kk G_ll
    k2 = (np.asarray(qtab, dtype=np.int64) ** 2) * gg
    ay = np.abs(y)
    n = np.floor(ay / (qtab * np.sqrt(gg)) + 0.5).astype(np.int64)
    lhs = 4 * ay * ay
    for _ in range(3):
        up = lhs >= (2 * n + 1) ** 2 * k2          # round(|z|) >= n + 1
        n = np.where(up, n + 1, n)
        down = (n > 0) & (lhs < (2 * n - 1) ** 2 * k2)  # round(|z|) < n
        n = np.where(down, n - 1, n)
    return np.sign(y) * n


# ---------------------------------------------------------------------------
# Inverse (Section 3 inverts the kept coefficients; C_orth^-1 = C_orth^T, Section 2)
# ---------------------------------------------------------------------------


def inverse_orth(z: np.ndarray) -> np.ndarray:
    """A' = C_orth^T Z' C_orth in float64 for a stack of coefficient blocks."""
    t = approx_dct()
    return np.matmul(np.matmul(t.T, np.asarray(z, dtype=np.float64)), t)


def d_prime() -> np.ndarray:
    """d'_k = 24 / G_kk, so that S^2 = diag(d') / 24 (G = C0 C0^T is diagonal)."""
    g = np.diag(gram())
    d = 24 // g
    assert np.all(d * g == 24)
    return d


def retention_numerator(y: np.ndarray, r: int) -> np.ndarray:
    """R = C0^T D' (M_r . Y) D' C0 in exact int64, with D' = diag(d').

    Because S^2 = D'/24, the reconstruction C_orth^T (M_r . Z) C_orth equals
    R / 576 exactly, so R is the exact integer numerator of the inverse."""
    c0 = round_off_matrix()
    dp = np.diag(d_prime())
    ym = np.asarray(y, dtype=np.int64) * retention_mask(r)
    return np.matmul(np.matmul(c0.T, np.matmul(np.matmul(dp, ym), dp)), c0)


def dequantize(q: np.ndarray, qtab: np.ndarray) -> np.ndarray:
    """Z' = q . Q (the dequantised C_orth coefficients)."""
    return np.asarray(q, dtype=np.float64) * np.asarray(qtab, dtype=np.float64)


# ---------------------------------------------------------------------------
# Metrics (Section 3: PSNR; also MSE)
# ---------------------------------------------------------------------------


def mse_from_sse(sse: float, n_pixels: int) -> float:
    return float(sse) / float(n_pixels)


def psnr_from_mse(mse: float, peak: float = 255.0) -> float:
    """PSNR = 10 log10(peak^2 / MSE), +inf when MSE = 0."""
    if mse == 0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)


def average_psnr(values) -> float:
    """Average PSNR over images: the arithmetic mean of per-image dB (Section 3)."""
    v = np.asarray(list(values), dtype=np.float64)
    return float(np.mean(v))


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("np", "sqrtm", "annotations")]
