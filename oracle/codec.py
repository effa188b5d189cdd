"""Codec output of the keep-r / quantisation procedure.

Test infrastructure only (see the package docstring).

Section 3 keeps the r initial zig-zag coefficients of every block and sets the
rest to zero; a codec stores exactly those coefficients and shows the
reconstruction as 8-bit pixels.  Readings where the paper is silent (each is
listed in the design notes):
  * Storage of a block: its kept coefficients in zig-zag order as (run, value)
    pairs, run = number of zeros before a non-zero value; zeros after the last
    non-zero value produce no pair (the end of the block is implied by the
    pair count).  Kept coefficients: ranks 0 .. r-1 of Y for the zig-zag
    selection, all 64 quantised values q for the quantisation path.  The DC
    value is coded like the others (no prediction between blocks).
  * 8-bit reconstruction: clamp(round(A'), 0, 255) with round-half-away-from-
    zero (Matlab's round, as for C0).  For the zig-zag selection A' = R / 576
    with the integer numerator R, so the rounding is decided exactly as
    floor((R + 288) / 576).
"""
from __future__ import annotations

import numpy as np

from . import image, rdct


def rle_encode(values) -> list[tuple[int, int]]:
    """(run, value) pairs of a sequence in scan order; trailing zeros dropped."""
    pairs = []
    run = 0
    for v in values:
        v = int(v)
        if v == 0:
            run += 1
        else:
            pairs.append((run, v))
            run = 0
    return pairs


def rle_decode(pairs, n: int) -> np.ndarray:
    """Inverse of rle_encode for a sequence of length n."""
    out = np.zeros(n, dtype=np.int64)
    pos = 0
    for run, v in pairs:
        pos += int(run)
        out[pos] = v
        pos += 1
    if pos > n:
        raise ValueError("pairs overrun the block")
    return out


def zigzag_scan(block: np.ndarray, n_kept: int) -> np.ndarray:
    """The first n_kept coefficients of an 8x8 block in zig-zag order."""
    order = rdct.zigzag_order()[:n_kept]
    return np.array([block[k, l] for (k, l) in order], dtype=np.int64)


def zigzag_unscan(seq: np.ndarray) -> np.ndarray:
    """8x8 block from its first len(seq) zig-zag coefficients (rest zero)."""
    block = np.zeros((8, 8), dtype=np.int64)
    for v, (k, l) in zip(seq, rdct.zigzag_order()):
        block[k, l] = v
    return block


def u8_from_numerator(r_num: np.ndarray) -> np.ndarray:
    """clamp(round(R / 576), 0, 255), round half away from zero, exactly."""
    r_num = np.asarray(r_num, dtype=np.int64)
    return np.clip((r_num + 288) // 576, 0, 255).astype(np.uint8)


def u8_from_float(a: np.ndarray) -> np.ndarray:
    """clamp(round(A'), 0, 255) of a float reconstruction."""
    return np.clip(rdct.matlab_round(a), 0, 255).astype(np.uint8)


def codec_encode(img: np.ndarray, mode: str, r: int = 64, quality: int = 50,
                 level_shift: int = 128) -> dict:
    """Pairs per block (raster block order), their counts, and the 8-bit
    reconstruction of one plane.  mode 'zigzag' (keep r) or 'quant'."""
    img = np.asarray(img)
    h, w = img.shape
    a = image.tile(img).astype(np.int64)
    nby, nbx = a.shape[:2]
    pairs = []
    if mode == "zigzag":
        y = rdct.forward_blocks(a)
        coefs, n_kept = y, r
        recon = image.untile(u8_from_numerator(rdct.retention_numerator(y, r)), h, w)
    elif mode == "quant":
        qt = rdct.quant_table(quality)
        y = rdct.forward_blocks(a, level_shift)
        q = rdct.quantize(y, qt)
        coefs, n_kept = q, 64
        rec = rdct.inverse_orth(rdct.dequantize(q, qt)) + level_shift
        recon = image.untile(u8_from_float(rec), h, w)
        out_float = image.untile(rec, h, w)
    else:
        raise ValueError(mode)
    for by in range(nby):
        for bx in range(nbx):
            pairs.append(rle_encode(zigzag_scan(coefs[by, bx], n_kept)))
    res = {"pairs": pairs, "counts": np.array([len(p) for p in pairs], dtype=np.int64),
           "recon_u8": recon, "coefs": coefs, "n_kept": n_kept}
    if mode == "quant":
        res["recon_float"] = out_float
    return res


def codec_decode_coefs(pairs, n_kept: int, nby: int, nbx: int) -> np.ndarray:
    """(nby, nbx, 8, 8) coefficient blocks from per-block pairs."""
    out = np.zeros((nby, nbx, 8, 8), dtype=np.int64)
    for i, p in enumerate(pairs):
        out[i // nbx, i % nbx] = zigzag_unscan(rle_decode(p, n_kept))
    return out


__all__ = ["rle_encode", "rle_decode", "zigzag_scan", "zigzag_unscan", "u8_from_numerator",
           "u8_from_float", "codec_encode", "codec_decode_coefs"]
