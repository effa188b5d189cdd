"""Image-level oracle: 8x8 tiling, compress/evaluate pipelines, sampled blocks.

Test infrastructure only (see the package docstring).

Section 3 divides each image into 8x8 sub-blocks, transforms each block, keeps
the r initial zig-zag coefficients, inverts the transform and measures
PSNR.  Readings where the paper is silent: planes whose sides are not multiples
of 8 are padded by replicating the last row and column, and every metric is
taken over the plane's own pixels only.  Coefficients are laid out block-major:
block (by, bx) holds 64 values in natural order k * 8 + l, blocks in raster order.
"""
from __future__ import annotations

import numpy as np

from . import rdct

B = rdct.N


def n_blocks(height: int, width: int) -> tuple[int, int]:
    return (height + B - 1) // B, (width + B - 1) // B


def tile(img: np.ndarray) -> np.ndarray:
    """(H, W) plane -> (nby, nbx, 8, 8) blocks, edge-replicating partial blocks."""
    img = np.asarray(img)
    h, w = img.shape
    nby, nbx = n_blocks(h, w)
    ys = np.minimum(np.arange(nby * B), h - 1)
    xs = np.minimum(np.arange(nbx * B), w - 1)
    padded = img[ys][:, xs]
    return padded.reshape(nby, B, nbx, B).transpose(0, 2, 1, 3)


def untile(blocks: np.ndarray, height: int, width: int) -> np.ndarray:
    """(nby, nbx, 8, 8) -> (H, W), cropping the padding."""
    nby, nbx = blocks.shape[:2]
    full = blocks.transpose(0, 2, 1, 3).reshape(nby * B, nbx * B)
    return full[:height, :width]


def valid_mask(height: int, width: int) -> np.ndarray:
    """(nby, nbx, 8, 8) mask of pixels inside the plane."""
    nby, nbx = n_blocks(height, width)
    yy = np.arange(nby * B)[:, None] < height
    xx = np.arange(nbx * B)[None, :] < width
    m = (yy & xx).astype(np.int64)
    return m.reshape(nby, B, nbx, B).transpose(0, 2, 1, 3)


def block_major(coef_blocks: np.ndarray) -> np.ndarray:
    """(nby, nbx, 8, 8) -> flat block-major array (nby * nbx * 64)."""
    return np.ascontiguousarray(coef_blocks).reshape(-1)


# ---------------------------------------------------------------------------
# Pipelines
# ---------------------------------------------------------------------------


def forward_image(img: np.ndarray, level_shift: int = 0) -> np.ndarray:
    """Y blocks (nby, nbx, 8, 8) int64 of a plane (Section 3)."""
    return rdct.forward_blocks(tile(img), level_shift)


def retention_eval(img: np.ndarray, r_values, recon_r: int | None = None) -> dict:
    """Keep-r evaluation of one plane (Section 3).

    For every r in `r_values`: A'_r = C_orth^T (M_r . Z) C_orth, computed exactly
    as R_r / 576 with the integer numerator R_r; sse_num[r] = sum over the plane's
    pixels of (576 A - R_r)^2 (exact, units of 1/576^2), sse = sse_num / 576^2,
    and PSNR.  Returns Y, Z restricted to recon_r (if given), the reconstruction
    at recon_r and the per-r metrics."""
    img = np.asarray(img)
    h, w = img.shape
    a = tile(img).astype(np.int64)
    y = rdct.forward_blocks(a)
    vm = valid_mask(h, w)
    out = {"Y": y, "sse_num": {}, "sse": {}, "mse": {}, "psnr": {}}
    for r in r_values:
        num = rdct.retention_numerator(y, r)
        e = (576 * a - num) * vm
        s = int(np.sum(e * e))
        out["sse_num"][r] = s
        out["sse"][r] = s / 576.0 ** 2
        out["mse"][r] = rdct.mse_from_sse(out["sse"][r], h * w)
        out["psnr"][r] = rdct.psnr_from_mse(out["mse"][r])
    if recon_r is not None:
        num = rdct.retention_numerator(y, recon_r)
        out["R"] = num
        out["recon"] = untile(num / 576.0, h, w)
        out["Z"] = rdct.scale_coeffs(y) * rdct.retention_mask(recon_r)
    return out


def quant_eval(img: np.ndarray, qtab: np.ndarray, level_shift: int = 128) -> dict:
    """Quantise/dequantise evaluation of one plane: Y of the level-shifted blocks,
    q = round(Z / Q) exactly, A' = C_orth^T (q . Q) C_orth + shift in float64,
    SSE/MSE/PSNR over the plane's pixels."""
    img = np.asarray(img)
    h, w = img.shape
    a = tile(img).astype(np.int64)
    y = rdct.forward_blocks(a, level_shift)
    q = rdct.quantize(y, qtab)
    rec = rdct.inverse_orth(rdct.dequantize(q, qtab)) + level_shift
    vm = valid_mask(h, w)
    e = (a - rec) * vm
    sse = float(np.sum(e * e))
    mse = rdct.mse_from_sse(sse, h * w)
    return {"Y": y, "q": q, "recon_blocks": rec, "recon": untile(rec, h, w),
            "sse": sse, "mse": mse, "psnr": rdct.psnr_from_mse(mse)}


def quant_block_sse(img: np.ndarray, qtab: np.ndarray, level_shift: int = 128) -> np.ndarray:
    """Per-block SSE (nby, nbx) of the quantisation path, float64."""
    img = np.asarray(img)
    h, w = img.shape
    a = tile(img).astype(np.int64)
    y = rdct.forward_blocks(a, level_shift)
    q = rdct.quantize(y, qtab)
    rec = rdct.inverse_orth(rdct.dequantize(q, qtab)) + level_shift
    e = (a - rec) * valid_mask(h, w)
    return np.sum(e * e, axis=(2, 3))


# ---------------------------------------------------------------------------
# Sampled blocks (for planes too large to process whole)
# ---------------------------------------------------------------------------


def sample_blocks(img: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """8x8 blocks at block-major indices `idx` of a plane, edge-replicated."""
    img = np.asarray(img)
    h, w = img.shape
    nby, nbx = n_blocks(h, w)
    idx = np.asarray(idx, dtype=np.int64)
    by, bx = idx // nbx, idx % nbx
    ys = np.minimum(by[:, None] * B + np.arange(B)[None, :], h - 1)
    xs = np.minimum(bx[:, None] * B + np.arange(B)[None, :], w - 1)
    return img[ys[:, :, None], xs[:, None, :]]


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("np", "rdct", "annotations")]
