"""Comparison transforms and image-quality metrics.

Test infrastructure only (see the package docstring).

Section 3 evaluates the approximation with the keep-r procedure against other
transforms: the average PSNR, and the average UQI and MSE given as absolute
percentage errors (APE) relative to the exact DCT.  Section 2 introduces the
signed DCT (SDCT) as the main comparator, and Section 4 suggests floor and
ceiling in place of the round-off.  Every transform here is an 8x8 matrix T
applied to each block as T A T^T (Section 3); the inverse is
A' = T^-1 (M_r . Y) T^-T, which is T^T (M_r . Y) T for the orthogonal ones.

Transforms:
  dct        T = C, the exact DCT.
  rdct       T = C_orth = S C0 with C0 = [2 C] (the proposed approximation).
  sdct       T = sign(C) / sqrt(8).  Not orthogonal, so the inverse is the
             matrix inverse.
  rdct_ceil  C0 = ceil(2 C), T = (C0 C0^T)^(-1/2) C0: the polar-decomposition
             construction of Section 2 applied to the ceiling.  C0 C0^T is not
             diagonal here, so S is a full matrix.
  rdct_floor C0 = floor(2 C).  Its first row (DC) is zero, C0 C0^T is singular
             and no orthogonal approximation exists; transform() raises.

Readings where the paper is silent (each is listed in the design notes):
  * UQI is Wang and Bovik's universal quality index,
        Q = 4 s_xy xbar ybar / ((s_x^2 + s_y^2)(xbar^2 + ybar^2)),
    evaluated as the product of f_s = 2 s_xy / (s_x^2 + s_y^2) and
    f_m = 2 xbar ybar / (xbar^2 + ybar^2).  Each factor is taken as 1 when its
    denominator is 0 (both windows flat, or both means zero).  The window is 8x8,
    sliding with stride 1 over the plane, (H - 7)(W - 7) windows; an image's UQI
    is the mean over its windows.
  * Float64 noise must not decide the index.  A constant block keeps only its
    DC term and is reconstructed exactly in real arithmetic, but the float64
    transforms leave ~1e-13 of noise in it; in a flat or all-zero area that noise
    alone would then set f_s or f_m.  So, in grey levels: a reconstruction window
    whose variance (over N = 64 pixels) is at most 2^-32 counts as flat (s_y^2 =
    s_xy = 0), a window mean |ybar| <= 2^-32 counts as 0, and a flat pixel window
    has s_xy = 0.  Float64 noise (~1e-13 per pixel) stays more than three orders
    of magnitude below these bounds, and the bounds stay below the resolution of
    the integer-numerator reconstructions (a window whose numerators y d are not
    all equal has N^2 d^2 var >= N - 1, i.e. var >= 63 / (4096 d^2) >= 4.6e-8 for
    d <= 576; a nonzero numerator sum is at least 1, a mean of 1 / (64 d)), so for
    those the rules only ever apply to windows that are exactly flat or exactly
    zero-mean: the index itself.
  * The reconstruction is real-valued (no rounding or clipping), as for PSNR.
  * APE(m) = 100 |m_T - m_DCT| / |m_DCT|, on the averages over images.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import sqrtm

from . import image, rdct

TRANSFORMS = ("rdct", "dct", "sdct", "rdct_ceil", "rdct_floor")


def _polar_orthogonal(c0: np.ndarray) -> np.ndarray:
    """(C0 C0^T)^(-1/2) C0 with the principal square root (Section 2)."""
    g = (c0 @ c0.T).astype(np.float64)
    if abs(np.linalg.det(g)) < 0.5:      # integer Gram matrix: singular iff det == 0
        raise ValueError("C0 C0^T is singular: no orthogonal approximation")
    s = np.real_if_close(sqrtm(np.linalg.inv(g))).astype(np.float64)
    return s @ c0.astype(np.float64)


def round_variant_matrix(kind: str) -> np.ndarray:
    """Integer matrix op(2 C) for op in {round (Matlab's), floor, ceil}."""
    twoc = 2.0 * rdct.dct_matrix()
    if kind == "round":
        return rdct.matlab_round(twoc).astype(np.int64)
    if kind == "floor":
        return np.floor(twoc).astype(np.int64)
    if kind == "ceil":
        return np.ceil(twoc).astype(np.int64)
    raise ValueError(kind)


def transform(name: str) -> tuple[np.ndarray, np.ndarray]:
    """(T, T^-1) in float64 for a transform name (see the module docstring)."""
    if name == "dct":
        t = rdct.dct_matrix()
        return t, t.T.copy()
    if name == "rdct":
        t = rdct.approx_dct()
        return t, t.T.copy()
    if name == "sdct":
        t = np.sign(rdct.dct_matrix()) / np.sqrt(8.0)
        return t, np.linalg.inv(t)
    if name == "rdct_ceil":
        t = _polar_orthogonal(round_variant_matrix("ceil"))
        return t, t.T.copy()
    if name == "rdct_floor":
        t = _polar_orthogonal(round_variant_matrix("floor"))   # raises
        return t, t.T.copy()
    raise ValueError(f"unknown transform {name!r}")


def sdct_integer_inverse() -> np.ndarray:
    """M = 8 sign(C)^-1, an integer matrix: the SDCT inverse is M / sqrt(8), so
    the keep-r reconstruction is A' = M (M_r . P) M^T / 64 with the integer
    P = sign(C) A sign(C)^T.  Asserts that 8 sign(C)^-1 is integral."""
    sgn = np.sign(rdct.dct_matrix())
    m = 8.0 * np.linalg.inv(sgn)
    mi = np.rint(m).astype(np.int64)
    assert np.max(np.abs(m - mi)) < 1e-9
    assert np.array_equal(mi @ sgn.astype(np.int64), 8 * np.eye(8, dtype=np.int64))
    return mi


# ---------------------------------------------------------------------------
# Keep-r reconstruction (Section 3) for any transform
# ---------------------------------------------------------------------------


def retention_recon(img: np.ndarray, name: str, r: int) -> np.ndarray:
    """A' (H, W) float64: every 8x8 block A -> Y = T A T^T, keep the r initial
    zig-zag coefficients, A' = T^-1 (M_r . Y) T^-T (Section 3)."""
    img = np.asarray(img)
    h, w = img.shape
    t, ti = transform(name)
    a = image.tile(img).astype(np.float64)
    y = np.matmul(np.matmul(t, a), t.T)
    y = y * rdct.retention_mask(r)
    rec = np.matmul(np.matmul(ti, y), ti.T)
    return image.untile(rec, h, w)


def sdct_numerators(img: np.ndarray, r: int) -> np.ndarray:
    """Exact integer N (H, W) with A'_sdct = N / 64 (see sdct_integer_inverse)."""
    img = np.asarray(img)
    h, w = img.shape
    sgn = np.sign(rdct.dct_matrix()).astype(np.int64)
    m = sdct_integer_inverse()
    a = image.tile(img).astype(np.int64)
    p = np.matmul(np.matmul(sgn, a), sgn.T) * rdct.retention_mask(r)
    return image.untile(np.matmul(np.matmul(m, p), m.T), h, w)


# ---------------------------------------------------------------------------
# UQI (universal quality index) over 8x8 sliding windows
# ---------------------------------------------------------------------------

WIN = 8
FLAT_EPS = 2.0 ** -32


def uqi_map(x: np.ndarray, y: np.ndarray, win: int = WIN) -> np.ndarray:
    """Q of every win x win window (stride 1) of two equally sized planes:
    ((H - win + 1), (W - win + 1)) float64."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape or min(x.shape) < win:
        raise ValueError("planes must match and hold at least one window")
    xw = np.lib.stride_tricks.sliding_window_view(x, (win, win))
    yw = np.lib.stride_tricks.sliding_window_view(y, (win, win))
    mx = xw.mean(axis=(2, 3))
    my = yw.mean(axis=(2, 3))
    dx = xw - mx[..., None, None]
    dy = yw - my[..., None, None]
    n1 = win * win - 1
    vx = (dx * dx).sum(axis=(2, 3)) / n1
    vy = (dy * dy).sum(axis=(2, 3)) / n1
    cxy = (dx * dy).sum(axis=(2, 3)) / n1
    flat_x = vx == 0
    flat_y = vy * n1 / (win * win) <= FLAT_EPS
    vy = np.where(flat_y, 0.0, vy)
    cxy = np.where(flat_x | flat_y, 0.0, cxy)
    my = np.where(np.abs(my) <= FLAT_EPS, 0.0, my)
    den_s = vx + vy
    den_m = mx * mx + my * my
    with np.errstate(divide="ignore", invalid="ignore"):
        f_s = np.where(den_s == 0, 1.0, 2.0 * cxy / den_s)
        f_m = np.where(den_m == 0, 1.0, 2.0 * mx * my / den_m)
    return f_s * f_m


def uqi(x: np.ndarray, y: np.ndarray, win: int = WIN) -> float:
    """Mean UQI over all win x win windows."""
    return float(np.mean(uqi_map(x, y, win)))


def uqi_map_exact(x: np.ndarray, y_num: np.ndarray, d: int, win: int = WIN) -> np.ndarray:
    """Q of every window for integer pixels x and a reconstruction given as
    integer numerators y = y_num / d.  The window sums are exact (int64); the
    degenerate-denominator rule is decided on exact integers, and only the
    final two divisions round.  Same definition as uqi_map, with s_xy, s_x^2,
    s_y^2 and the means written over N^2 d^2 as integer expressions."""
    x = np.asarray(x, dtype=np.int64)
    yn = np.asarray(y_num, dtype=np.int64)
    n = win * win
    sw = np.lib.stride_tricks.sliding_window_view

    def wsum(a):
        return sw(a, (win, win)).sum(axis=(2, 3))
    sx, sxx = wsum(x), wsum(x * x)
    sy, syy, sxy = wsum(yn), wsum(yn * yn), wsum(x * yn)
    vx = n * sxx - sx * sx
    vy = n * syy - sy * sy                    # n^2 d^2 var_y
    # The flat-window rules on exact integers (the bounds n^2 d^2 2^-32 and
    # n d 2^-32 are exact in float64; below the integers' resolution, so they
    # hold only for exactly flat or exactly zero-mean windows).
    flat_y = vy.astype(np.float64) <= n * n * d * d * FLAT_EPS
    vy = np.where(flat_y, 0, vy)
    cov = np.where((vx == 0) | flat_y, 0, n * sxy - sx * sy)
    sy = np.where(np.abs(sy).astype(np.float64) <= n * d * FLAT_EPS, 0, sy)
    num_s = 2 * d * cov
    den_s = d * d * vx + vy
    num_m = 2 * d * sx * sy
    den_m = d * d * sx * sx + sy * sy
    with np.errstate(divide="ignore", invalid="ignore"):
        f_s = np.where(den_s == 0, 1.0, num_s.astype(np.float64) / den_s.astype(np.float64))
        f_m = np.where(den_m == 0, 1.0, num_m.astype(np.float64) / den_m.astype(np.float64))
    return f_s * f_m


def integer_numerators(img: np.ndarray, name: str, r: int) -> tuple[np.ndarray, int]:
    """(numerator plane, d) of the keep-r reconstruction for the transforms whose
    reconstruction is an integer over a fixed d: rdct (R / 576) and sdct (N / 64)."""
    if name == "rdct":
        h, w = np.asarray(img).shape
        y = rdct.forward_blocks(image.tile(img))
        return image.untile(rdct.retention_numerator(y, r), h, w), 576
    if name == "sdct":
        return sdct_numerators(img, r), 64
    raise ValueError(f"{name} has no integer numerator")


def uqi_window_exact(xw, yw):
    """Q of one window with exact rational arithmetic (fractions.Fraction);
    brute-force pin for small cases."""
    from fractions import Fraction
    xs = [Fraction(v) for v in np.asarray(xw).ravel().tolist()]
    ys = [Fraction(v) for v in np.asarray(yw).ravel().tolist()]
    n = len(xs)
    mx = sum(xs) / n
    my = sum(ys) / n
    vx = sum((v - mx) ** 2 for v in xs) / (n - 1)
    vy = sum((v - my) ** 2 for v in ys) / (n - 1)
    cxy = sum((a - mx) * (b - my) for a, b in zip(xs, ys)) / (n - 1)
    flat_y = vy * (n - 1) / n <= Fraction(FLAT_EPS)
    if flat_y:
        vy = Fraction(0)
    if vx == 0 or flat_y:
        cxy = Fraction(0)
    if abs(my) <= Fraction(FLAT_EPS):
        my = Fraction(0)
    f_s = Fraction(1) if vx + vy == 0 else 2 * cxy / (vx + vy)
    f_m = Fraction(1) if mx * mx + my * my == 0 else 2 * mx * my / (mx * mx + my * my)
    return f_s * f_m


# ---------------------------------------------------------------------------
# Per-image sweep and the APE of Section 3
# ---------------------------------------------------------------------------


def quality_eval(img: np.ndarray, name: str, r_values) -> dict:
    """For each r: SSE, MSE, PSNR and mean UQI of the keep-r reconstruction of
    one plane under transform `name`."""
    img = np.asarray(img)
    h, w = img.shape
    x = img.astype(np.float64)
    out = {"sse": {}, "mse": {}, "psnr": {}, "uqi": {}}
    for r in r_values:
        rec = retention_recon(img, name, r)
        e = x - rec
        sse = float(np.sum(e * e))
        out["sse"][r] = sse
        out["mse"][r] = rdct.mse_from_sse(sse, h * w)
        out["psnr"][r] = rdct.psnr_from_mse(out["mse"][r])
        out["uqi"][r] = uqi(x, rec)
    return out


def ape(value: float, reference: float) -> float:
    """Absolute percentage error of a metric relative to the exact DCT's."""
    return 100.0 * abs(value - reference) / abs(reference)


__all__ = ["TRANSFORMS", "round_variant_matrix", "transform", "sdct_integer_inverse",
           "retention_recon", "sdct_numerators", "uqi_map", "uqi", "uqi_map_exact",
           "integer_numerators", "uqi_window_exact", "quality_eval", "ape", "WIN"]
